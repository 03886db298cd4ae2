// The diffusion operator of the monodomain step applied on its own to a
// caller's potential field: node values by inverse-distance weights, then
// the face-flux sum of every cell (Sec. 3.2: node interpolation, cell
// gradients, face gradients of eq. gra2bis, the finite-volume flux sum),
// through the same device functions as the fused step kernel, so the result
// equals the L the step computes from the same v^n.
//
// Three kernels over plain grids of 256 lanes: the caller's v (caller order,
// FP64) is gathered into internal order in the working precision, the node
// values are formed, and the flux sum of each cell is scattered back to
// caller order in FP64.  The workspace holds the internal-order potentials
// and the node values.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "instance.hpp"
#include "kernels.hpp"

namespace ep {
namespace {

using epdev::InstDesc;

template <typename R>
__global__ void __launch_bounds__(256) k_diff_in(const double *__restrict__ v,
                                                  const int32_t *__restrict__ perm,
                                                  R *__restrict__ vi, int64_t nc) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c < nc) vi[c] = R(v[perm[c]]);
}

// node tiles in the chunked XCD ranges of the step's node gather
// (neighbouring node tiles share cells, whose potentials then stay in one L2)
template <typename R>
__global__ void __launch_bounds__(256) k_diff_nodes(InstDesc D, const R *__restrict__ vi,
                                                     R *__restrict__ vn) {
    const int64_t tile = epdev::chunk_tile(epdev::xcd_tile(blockIdx.x, gridDim.x), gridDim.x);
    const int64_t node = tile * 256 + threadIdx.x;
    if (node < D.nn) vn[node] = epdev::node_value<R>(D, node, vi);
}

template <typename R>
__global__ void __launch_bounds__(256) k_diff_out(InstDesc D, const R *__restrict__ vi,
                                                   const R *__restrict__ vn,
                                                   const int32_t *__restrict__ perm,
                                                   double *__restrict__ L) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c < D.nc) {
        const uint32_t cc = (uint32_t)c;
        L[perm[c]] = double(epdev::flux_sum<R, false>(D, cc, vi, vn, vi[c]));
    }
}

template <typename R>
std::string launch(const Inst &I, hipStream_t st, const double *v, double *L, void *ws) {
    const int64_t nc = I.desc.nc, nn = I.desc.nn;
    R *vi = (R *)ws;
    R *vn = (R *)((char *)ws + diffusion_workspace_split(nc, sizeof(R)));
    const unsigned gc = (unsigned)((nc + 255) / 256), gn = (unsigned)((nn + 255) / 256);
    k_diff_in<R><<<gc, 256, 0, st>>>(v, I.d_perm, vi, nc);
    k_diff_nodes<R><<<gn, 256, 0, st>>>(I.desc, vi, vn);
    k_diff_out<R><<<gc, 256, 0, st>>>(I.desc, vi, vn, I.d_perm, L);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? std::string() : std::string("diffusion kernels: ") + hipGetErrorString(e);
}

// Fixed workspace of the no-allocation entry point, one copy per GPU for the
// life of the process.  Host code never takes the array's own name as an
// address: it uses the device address hipGetSymbolAddress gives for the
// current device (g_scratch).
constexpr size_t kScratchBytes = (size_t)EP_DIFFUSION_SCRATCH_MAX;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

}  // namespace

size_t diffusion_workspace_split(int64_t nc, size_t rs) {
    return ((size_t)nc * rs + 255) / 256 * 256;
}

size_t diffusion_workspace_bytes(const Inst &I) {
    return diffusion_workspace_split(I.desc.nc, (size_t)I.rs) + (size_t)I.desc.nn * (size_t)I.rs;
}

std::string diffusion_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return "device index beyond the scratch table";
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return "";
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // device is current
    if (e != hipSuccess) return std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    g_scratch[device] = p;
    return "";
}

std::string diffusion_apply(const Inst &I, hipStream_t st, const double *v, double *L, void *ws) {
    return I.rs == 8 ? launch<double>(I, st, v, L, ws) : launch<float>(I, st, v, L, ws);
}

std::string diffusion_apply_noalloc(const Inst &I, int device, hipStream_t st, const double *v,
                                    double *L, ep_status &code) {
    const size_t need = diffusion_workspace_bytes(I);
    if (need > kScratchBytes) {
        code = EP_EINVAL;
        return "the operator needs " + std::to_string(need) +
               " bytes of workspace; the fixed buffer holds " + std::to_string(kScratchBytes);
    }
    void *p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (device >= 0 && device < kMaxDevices) p = g_scratch[device];
    }
    if (!p) {
        code = EP_ESTATE;
        return "no workspace address for this device (taken at ep_init)";
    }
    code = EP_EDEVICE;
    return diffusion_apply(I, st, v, L, p);
}

}  // namespace ep
