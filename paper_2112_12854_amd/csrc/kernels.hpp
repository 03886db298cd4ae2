// Device kernels of the monodomain step.
//
// Per step two kernels run: the node gather (the inverse-distance node
// values of Sec. 3.2) and the fused cell kernel, which evaluates the face
// fluxes from the node values and neighbour potentials, the stimulus, the
// cell model, v^{n+1} = v^n + dt (L - I_ion - I_stim) and the activation /
// APD90 detection, all with level-n inputs.  Cells and nodes are
// renumbered on the host so that a block's gathers are local; both kernels
// read structure-of-arrays data with consecutive lanes on consecutive
// entries.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "cellmodels.hpp"

namespace epdev {

constexpr int MAX_STIM = 32;
constexpr int NG_MAX = 15;   // gate slots (CRN)
constexpr int NC_MAX = 6;    // FP64 slots (Stewart)

// Device-resident control block: read by every kernel of a step, so a
// captured graph can be replayed at any step index.
struct Ctrl {
    int64_t step;                 // index n of the next step
    int32_t nan_flag;             // set when a non-finite v^{n+1} appears
    int32_t n_stim;
    int64_t st_n0[MAX_STIM];      // first active step
    int64_t st_ndur[MAX_STIM];    // active steps per pulse
    int64_t st_nper[MAX_STIM];    // steps between pulses (0 = single pulse)
    int32_t st_count[MAX_STIM];   // pulses
    double st_amp[MAX_STIM];      // pA/pF
};

// Map block b of nb so that each of the 8 XCDs (blocks are dealt round-robin
// to XCDs) works on one contiguous range of tiles and its L2 sees the
// neighbour data of its own range.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
    const int64_t x = b & 7, i = b >> 3;
    const int64_t q = nb >> 3, r = nb & 7;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

template <typename R>
__global__ void k_node_gather(int64_t nn, const int64_t *__restrict__ off,
                              const int32_t *__restrict__ cell,
                              const R *__restrict__ w, const R *__restrict__ v,
                              R *__restrict__ vn, int remap) {
    const int64_t b = remap ? xcd_tile(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int64_t n = b * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const int64_t lane = n & 63;
    const int64_t e0 = off[n >> 6] + lane, e1 = off[(n >> 6) + 1];
    // four independent gathers in flight per lane; the sum order is fixed
    R a0 = R(0), a1 = R(0), a2 = R(0), a3 = R(0);
    int64_t e = e0;
    for (; e + 192 < e1; e += 256) {
        const int32_t c0 = cell[e], c1 = cell[e + 64], c2 = cell[e + 128], c3 = cell[e + 192];
        const R w0 = w[e], w1 = w[e + 64], w2 = w[e + 128], w3 = w[e + 192];
        a0 += w0 * v[c0];
        a1 += w1 * v[c1];
        a2 += w2 * v[c2];
        a3 += w3 * v[c3];
    }
    for (; e < e1; e += 64) a0 += w[e] * v[cell[e]];
    vn[n] = (a0 + a1) + (a2 + a3);
}

template <typename R>
struct CellArgs {
    int64_t n;                               // cells
    const int32_t *__restrict__ cnode;       // [8][n]
    const R *__restrict__ cbeta;             // [8][n]
    const int32_t *__restrict__ cnbr;        // [4][n]
    const R *__restrict__ cb;                // [4][n]
    const R *__restrict__ vn;                // node values
    const R *__restrict__ vin;               // v^n
    R *__restrict__ vout;                    // v^{n+1}
    R *__restrict__ gate;                    // [NG_MAX][n]
    double *__restrict__ conc;               // [NC_MAX][n]
    const uint8_t *__restrict__ model;       // [n]
    const uint32_t *__restrict__ smask;      // [n] stimulus membership bits
    uint8_t *__restrict__ dstat;             // 0 resting, 1 activated, 2 repolarised
    double *__restrict__ t_act;
    double *__restrict__ t_rep;
    R *__restrict__ vmax;
    const R *__restrict__ vrest;
    Ctrl *ctrl;
    R dt;
    double dtd;
    R thr, repol;
    GScale gs;
};

// MSET: bit 0 TP06 (any layer), 1 CRN, 2 Stewart, 3 passive.
template <typename R, int MSET>
__global__ void __launch_bounds__(256) k_cell(CellArgs<R> a, int32_t step_off, int remap) {
    const int64_t b = remap ? xcd_tile(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int64_t c = b * blockDim.x + threadIdx.x;
    const int64_t N = a.n;
    const int64_t n = a.ctrl->step + step_off;
    const int ns = a.ctrl->n_stim;
    uint32_t active = 0;
    for (int i = 0; i < ns; ++i) {
        const int64_t k = n - a.ctrl->st_n0[i];
        const int64_t per = a.ctrl->st_nper[i];
        bool on = k >= 0 && (per <= 0 ? k < a.ctrl->st_ndur[i]
                                      : (k / per) < a.ctrl->st_count[i] &&
                                            (k % per) < a.ctrl->st_ndur[i]);
        active |= (on ? 1u : 0u) << i;
    }
    if (c >= N) return;

    // ---- diffusion: fused node-coefficient stencil plus two-point terms
    const R v = a.vin[c];
    R L = R(0);
#pragma unroll
    for (int s = 0; s < 8; ++s) L += a.cbeta[s * N + c] * a.vn[a.cnode[s * N + c]];
#pragma unroll
    for (int f = 0; f < 4; ++f) L += a.cb[f * N + c] * (a.vin[a.cnbr[f * N + c]] - v);

    // ---- stimulus
    R istim = R(0);
    if (active) {
        uint32_t m = a.smask[c] & active;
        while (m) {
            const int i = __ffs(m) - 1;
            istim += R(a.ctrl->st_amp[i]);
            m &= m - 1;
        }
    }

    // ---- cell model
    R iion = R(0);
    const int md = (MSET == 8) ? 5 : a.model[c];   // TP06 layer or model id
    R g[NG_MAX];
    double cc[NC_MAX];
    if ((MSET & 1) && md <= 2) {
#pragma unroll
        for (int s = 0; s < tp06::NG; ++s) g[s] = a.gate[s * N + c];
#pragma unroll
        for (int s = 0; s < tp06::NC; ++s) cc[s] = a.conc[s * N + c];
        iion = tp06::step<R>(md, v, g, cc, a.dt, a.dtd, istim, a.gs);
#pragma unroll
        for (int s = 0; s < tp06::NG; ++s) a.gate[s * N + c] = g[s];
#pragma unroll
        for (int s = 0; s < tp06::NC; ++s) a.conc[s * N + c] = cc[s];
    } else if ((MSET & 2) && md == 3) {
#pragma unroll
        for (int s = 0; s < crn::NG; ++s) g[s] = a.gate[s * N + c];
#pragma unroll
        for (int s = 0; s < crn::NC; ++s) cc[s] = a.conc[s * N + c];
        iion = crn::step<R>(v, g, cc, a.dt, a.dtd, a.gs);
#pragma unroll
        for (int s = 0; s < crn::NG; ++s) a.gate[s * N + c] = g[s];
#pragma unroll
        for (int s = 0; s < crn::NC; ++s) a.conc[s * N + c] = cc[s];
    } else if ((MSET & 4) && md == 4) {
#pragma unroll
        for (int s = 0; s < stewart::NG; ++s) g[s] = a.gate[s * N + c];
#pragma unroll
        for (int s = 0; s < stewart::NC; ++s) cc[s] = a.conc[s * N + c];
        iion = stewart::step<R>(v, g, cc, a.dt, a.dtd, istim, a.gs);
#pragma unroll
        for (int s = 0; s < stewart::NG; ++s) a.gate[s * N + c] = g[s];
#pragma unroll
        for (int s = 0; s < stewart::NC; ++s) a.conc[s * N + c] = cc[s];
    }

    // ---- explicit update of v
    const R vnew = v + a.dt * (L - iion - istim);
    a.vout[c] = vnew;
    if (!(fabs(vnew) < R(1e30))) atomicOr(&a.ctrl->nan_flag, 1);

    // ---- activation time and APD90
    const uint8_t st = a.dstat[c];
    if (st == 0) {
        if (v <= a.thr && vnew > a.thr) {
            a.t_act[c] = (double(n) + double((a.thr - v) / (vnew - v))) * a.dtd;
            a.vmax[c] = vnew;
            a.dstat[c] = 1;
        }
    } else if (st == 1) {
        R vm = a.vmax[c];
        if (vnew > vm) {
            vm = vnew;
            a.vmax[c] = vm;
        }
        const R v90 = vm - a.repol * (vm - a.vrest[c]);
        if (v >= v90 && vnew < v90) {
            a.t_rep[c] = (double(n) + double((v - v90) / (v - vnew))) * a.dtd;
            a.dstat[c] = 2;
        }
    }
}

__global__ void k_advance(Ctrl *ctrl, int64_t k) { ctrl->step += k; }

// Volume-weighted sum of v, stage 1: one partial per block.
template <typename R>
__global__ void __launch_bounds__(256) k_vsum_partial(int64_t n, const R *__restrict__ v,
                                                      const double *__restrict__ vol,
                                                      double *__restrict__ part) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (int64_t)gridDim.x * 256)
        acc += vol[c] * double(v[c]);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Stage 2 (one block): fixed-order sum of the partials, stored as the trace
// sample of step ctrl->step + step_off.
__global__ void __launch_bounds__(256) k_vsum_final(int nparts, const double *__restrict__ part,
                                                    double inv_vol, const Ctrl *ctrl, int32_t step_off,
                                                    int32_t every, int64_t cap,
                                                    double *__restrict__ trace) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t idx = (ctrl->step + step_off) / every;
        if (idx >= 0 && idx < cap) trace[idx] = red[0] * inv_vol;
    }
}

}  // namespace epdev
