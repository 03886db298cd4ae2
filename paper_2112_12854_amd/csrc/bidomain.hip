// Extracellular solve of the bidomain step (Sec. 3.1 eq. electro, Sec. 3.2
// eq. electro2_3d): once v^{n+1} is known,
//   sum_f A_f ((M_i + M_e) grad phi).n_f = -sum_f A_f (M_i grad v^{n+1}).n_f
// is solved for phi_e^{n+1} by restarted GMRES from phi_e^n, on the device.
//
// The operator is the same node gather plus fused cell stencil as the time
// step, with the coefficients of M_i + M_e in flux-sum form.  The Arnoldi
// basis is orthogonalised by classical Gram-Schmidt applied twice (batched
// dot products instead of the j + 1 dependent passes of the modified
// variant); dot products are per-block partials added in a fixed order, so a
// solve gives the same bits on every run.  Only the (restart + 1) x restart
// Hessenberg least-squares problem (Givens rotations, back substitution) is
// advanced on the host, from a few numbers read back per Arnoldi step.
// GMRES is preconditioned on the right by a two-level additive method (the
// residual it monitors stays the true one): Jacobi plus a dense solve on
// aggregates of cells, which removes the growth of the iteration count with
// the grid size that the plain method shows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "instance.hpp"

namespace ep {

using epdev::InstDesc;
using epdev::tix;

namespace {

constexpr int BT = 256;        // threads per block
constexpr int NQ = 8;          // dot products per pass of the reduction kernel
constexpr int G = kBidoBlocks; // blocks of the reduction kernels

// node values by inverse-distance weights (sliced ELL, one lane per node)
__global__ void __launch_bounds__(BT) k_gather(const int64_t *__restrict__ off,
                                               const int32_t *__restrict__ cell,
                                               const double *__restrict__ w,
                                               const double *__restrict__ x,
                                               double *__restrict__ xn, int64_t nn) {
    const int64_t node = blockIdx.x * (int64_t)BT + threadIdx.x;
    if (node >= nn) return;
    const int64_t e0 = off[node >> 6] + (node & 63), e1 = off[(node >> 6) + 1];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t e = e0;
    for (; e + 192 < e1; e += 256) {
        a0 += w[e] * x[cell[e]];
        a1 += w[e + 64] * x[cell[e + 64]];
        a2 += w[e + 128] * x[cell[e + 128]];
        a3 += w[e + 192] * x[cell[e + 192]];
    }
    for (; e < e1; e += 64) a0 += w[e] * x[cell[e]];
    xn[node] = (a0 + a1) + (a2 + a3);
}

// y_c = f_c (sum_s beta_s x_n[node_s] + sum_f b_f (x[nbr_f] - x_c)) with the
// stencil in tile-major slot arrays,
// f_c = factor * V_c with a volume array, else factor
__global__ void __launch_bounds__(BT) k_flux(const int32_t *__restrict__ cnode,
                                             const double *__restrict__ beta,
                                             const int32_t *__restrict__ cnbr,
                                             const double *__restrict__ bf,
                                             const double *__restrict__ x,
                                             const double *__restrict__ xn,
                                             const double *__restrict__ vol, double factor,
                                             double *__restrict__ y, int64_t nc) {
    const int64_t c = blockIdx.x * (int64_t)BT + threadIdx.x;
    if (c >= nc) return;
    const double xc = x[c];
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < 8; ++s) acc += beta[tix(c, s, 8)] * xn[cnode[tix(c, s, 8)]];
#pragma unroll
    for (int f = 0; f < 4; ++f) acc += bf[tix(c, f, 4)] * (x[cnbr[tix(c, f, 4)]] - xc);
    y[c] = (vol ? factor * vol[c] : factor) * acc;
}

// per-block partial sums of cnt <= NQ dot products <w, V_q>, V_q = V + q n
__global__ void __launch_bounds__(BT) k_dots(const double *__restrict__ w,
                                             const double *__restrict__ V, int cnt, int64_t n,
                                             double *__restrict__ part) {
    __shared__ double red[NQ][BT];
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x; e < n; e += (int64_t)G * BT) {
        const double we = w[e];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (q < cnt) acc[q] += we * V[q * n + e];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int s = BT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int q = 0; q < cnt; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
        __syncthreads();
    }
    if ((int)threadIdx.x < cnt) part[(int64_t)threadIdx.x * G + blockIdx.x] = red[threadIdx.x][0];
}

// out[q] = sum of the G partials of row q (one block per row, fixed order)
__global__ void __launch_bounds__(BT) k_reduce(const double *__restrict__ part,
                                               double *__restrict__ out) {
    __shared__ double red[BT];
    const double *p = part + (int64_t)blockIdx.x * G;
    double acc = 0.0;
    for (int i = threadIdx.x; i < G; i += BT) acc += p[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = BT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// w -= sum_{q < cnt} h_q V_q
__global__ void __launch_bounds__(BT) k_sub(double *__restrict__ w, const double *__restrict__ V,
                                            const double *__restrict__ h, int cnt, int64_t n) {
    const int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x;
    if (e >= n) return;
    double x = w[e];
    for (int q = 0; q < cnt; ++q) x -= h[q] * V[q * n + e];
    w[e] = x;
}

// x += sum_{q < cnt} y_q V_q
__global__ void __launch_bounds__(BT) k_update(double *__restrict__ x, const double *__restrict__ V,
                                               const double *__restrict__ y, int cnt, int64_t n) {
    const int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x;
    if (e >= n) return;
    double acc = x[e];
    for (int q = 0; q < cnt; ++q) acc += y[q] * V[q * n + e];
    x[e] = acc;
}

// dst = a src
__global__ void __launch_bounds__(BT) k_scale(double *__restrict__ dst, const double *__restrict__ src,
                                              double a, int64_t n) {
    const int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x;
    if (e < n) dst[e] = a * src[e];
}

// w = b - w
__global__ void __launch_bounds__(BT) k_resid(double *__restrict__ w, const double *__restrict__ b,
                                              int64_t n) {
    const int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x;
    if (e < n) w[e] = b[e] - w[e];
}

// x -= s / total (s: device scalar)
__global__ void __launch_bounds__(BT) k_shift(double *__restrict__ x, const double *__restrict__ s,
                                              double inv_total, int64_t n) {
    const int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x;
    if (e < n) x[e] -= s[0] * inv_total;
}

// ---- two-level preconditioner z = omega D^{-1} r + P A_c^{-1} P^T r
// rc[I] = sum of r over aggregate I (one block per aggregate, fixed order)
__global__ void __launch_bounds__(BT) k_restrict(const double *__restrict__ r,
                                                 const int32_t *__restrict__ off,
                                                 const int32_t *__restrict__ cells,
                                                 double *__restrict__ rc) {
    __shared__ double red[BT];
    double acc = 0.0;
    for (int32_t i = off[blockIdx.x] + threadIdx.x; i < off[blockIdx.x + 1]; i += BT) acc += r[cells[i]];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = BT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) rc[blockIdx.x] = red[0];
}

// zc = A_c^{-1} rc (dense, row-major; one block per row)
__global__ void __launch_bounds__(BT) k_coarse(const double *__restrict__ cinv,
                                               const double *__restrict__ rc,
                                               double *__restrict__ zc, int32_t na) {
    __shared__ double red[BT];
    const double *row = cinv + (int64_t)blockIdx.x * na;
    double acc = 0.0;
    for (int32_t j = threadIdx.x; j < na; j += BT) acc += row[j] * rc[j];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = BT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) zc[blockIdx.x] = red[0];
}

// z = omega D^{-1} r + zc[aggregate]
__global__ void __launch_bounds__(BT) k_smooth(const double *__restrict__ r,
                                               const double *__restrict__ dinv,
                                               const int32_t *__restrict__ agg_of,
                                               const double *__restrict__ zc, double omega,
                                               double *__restrict__ z, int64_t n) {
    const int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x;
    if (e < n) z[e] = omega * dinv[e] * r[e] + zc[agg_of[e]];
}

// t = sum_{q < cnt} y_q V_q
__global__ void __launch_bounds__(BT) k_combine(double *__restrict__ t, const double *__restrict__ V,
                                                const double *__restrict__ y, int cnt, int64_t n) {
    const int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x;
    if (e >= n) return;
    double acc = 0.0;
    for (int q = 0; q < cnt; ++q) acc += y[q] * V[q * n + e];
    t[e] = acc;
}

// x += z
__global__ void __launch_bounds__(BT) k_add(double *__restrict__ x, const double *__restrict__ z,
                                            int64_t n) {
    const int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x;
    if (e < n) x[e] += z[e];
}

constexpr double kOmega = 0.7;   // Jacobi weight of the preconditioner

struct Solver {
    Inst &I;
    hipStream_t st;
    int64_t nc, nn;
    int grid_c, grid_n;

    // partial rows [row0, row0 + cnt) <- <w, V + q n>, then reduced into out[0..cnt)
    void dots(const double *w, const double *V, int cnt, double *out) {
        for (int q0 = 0; q0 < cnt; q0 += NQ) {
            const int k = std::min(NQ, cnt - q0);
            k_dots<<<G, BT, 0, st>>>(w, V + (int64_t)q0 * nc, k, nc, I.bd.part + (int64_t)q0 * G);
        }
        k_reduce<<<cnt, BT, 0, st>>>(I.bd.part, out);
    }
    // y = A x (elliptic operator, flux-sum form)
    void apply(const double *x, double *y) {
        const InstDesc &D = I.desc;
        k_gather<<<grid_n, BT, 0, st>>>(D.sell_off, D.sell_cell, (const double *)D.sell_w, x, I.bd.xn, nn);
        k_flux<<<grid_c, BT, 0, st>>>(D.cnode, I.bd.ebeta, D.cnbr, I.bd.eb, x, I.bd.xn, nullptr, 1.0, y, nc);
    }
    // z = M^{-1} r
    void prec(const double *r, double *z) {
        const Bido &B = I.bd;
        k_restrict<<<B.n_agg, BT, 0, st>>>(r, B.agg_off, B.agg_cells, B.rc);
        k_coarse<<<B.n_agg, BT, 0, st>>>(B.cinv, B.rc, B.zc, B.n_agg);
        k_smooth<<<grid_c, BT, 0, st>>>(r, B.dinv, B.agg_of, B.zc, kOmega, z, nc);
    }
    hipError_t read(const double *dev, int cnt) {
        hipError_t e = hipMemcpyAsync(I.bd.h_host, dev, cnt * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(st);
    }
};

}  // namespace

std::string bidomain_solve(Inst &I, hipStream_t st) {
    Bido &B = I.bd;
    const InstDesc &D = I.desc;
    Solver S{I, st, D.nc, D.nn, (int)((D.nc + BT - 1) / BT), (int)((D.nn + BT - 1) / BT)};
    const int64_t nc = D.nc;
    const int m = B.restart;
    const double *v = (const double *)D.v[I.host_step & 1];
    double *hd = B.h;                       // [0, m] pass 1, [m+1, 2m+1] pass 2, then norms
    double *const h_norm = B.h + 2 * (m + 1);
    hipError_t e;
    auto fail = [&](const char *what) { return std::string(what) + ": " + hipGetErrorString(e); };

    // right-hand side: -chi Cm V_c L_i(v) = -(flux sums of v with M_i)
    k_gather<<<S.grid_n, BT, 0, st>>>(D.sell_off, D.sell_cell, (const double *)D.sell_w, v, B.xn, D.nn);
    k_flux<<<S.grid_c, BT, 0, st>>>(D.cnode, (const double *)D.cbeta, D.cnbr, (const double *)D.cb, v,
                                    B.xn, D.vol, -B.chi_cm, B.b, nc);
    S.dots(B.b, B.b, 1, h_norm);
    if ((e = S.read(h_norm, 1)) != hipSuccess) return fail("bidomain readback");
    const double bnorm = std::sqrt(B.h_host[0]);
    int64_t it = 0;
    double relres = 0.0;
    if (bnorm == 0.0) {
        k_scale<<<S.grid_c, BT, 0, st>>>(B.phi, B.phi, 0.0, nc);
    } else {
        std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
        for (;;) {
            S.apply(B.phi, B.w);
            k_resid<<<S.grid_c, BT, 0, st>>>(B.w, B.b, nc);
            S.dots(B.w, B.w, 1, h_norm);
            if ((e = S.read(h_norm, 1)) != hipSuccess) return fail("bidomain readback");
            const double beta = std::sqrt(B.h_host[0]);
            relres = beta / bnorm;
            if (beta <= B.tol * bnorm || it >= B.max_iter) break;
            k_scale<<<S.grid_c, BT, 0, st>>>(B.V, B.w, 1.0 / beta, nc);
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            int k = 0;
            for (int j = 0; j < m && it < B.max_iter; ++j) {
                const double *vj = B.V + (int64_t)j * nc;
                if (B.precond) {                     // right preconditioning: A M^{-1} v_j
                    S.prec(vj, B.z);
                    S.apply(B.z, B.w);
                } else {
                    S.apply(vj, B.w);
                }
                // classical Gram-Schmidt, twice
                S.dots(B.w, B.V, j + 1, hd);
                k_sub<<<S.grid_c, BT, 0, st>>>(B.w, B.V, hd, j + 1, nc);
                S.dots(B.w, B.V, j + 1, hd + (m + 1));
                k_sub<<<S.grid_c, BT, 0, st>>>(B.w, B.V, hd + (m + 1), j + 1, nc);
                S.dots(B.w, B.w, 1, h_norm);
                if ((e = hipMemcpyAsync(B.h_host, hd, (2 * (m + 1) + 1) * sizeof(double),
                                        hipMemcpyDeviceToHost, st)) != hipSuccess ||
                    (e = hipStreamSynchronize(st)) != hipSuccess)
                    return fail("bidomain readback");
                for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = B.h_host[i] + B.h_host[m + 1 + i];
                const double hn = std::sqrt(B.h_host[2 * (m + 1)]);
                H[(size_t)(j + 1) * m + j] = hn;
                for (int i = 0; i < j; ++i) {       // earlier rotations
                    const double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
                    H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
                    H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
                }
                const double den = std::hypot(H[(size_t)j * m + j], H[(size_t)(j + 1) * m + j]);
                cs[j] = den > 0.0 ? H[(size_t)j * m + j] / den : 1.0;
                sn[j] = den > 0.0 ? H[(size_t)(j + 1) * m + j] / den : 0.0;
                H[(size_t)j * m + j] = den;
                H[(size_t)(j + 1) * m + j] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                ++it;
                k = j + 1;
                if (std::fabs(g[j + 1]) <= B.tol * bnorm || hn == 0.0) break;
                k_scale<<<S.grid_c, BT, 0, st>>>(B.V + (int64_t)(j + 1) * nc, B.w, 1.0 / hn, nc);
            }
            for (int i = k - 1; i >= 0; --i) {      // R y = g
                double acc = g[i];
                for (int l = i + 1; l < k; ++l) acc -= H[(size_t)i * m + l] * y[l];
                y[i] = acc / H[(size_t)i * m + i];
            }
            if ((e = hipMemcpyAsync(B.y, y.data(), k * sizeof(double), hipMemcpyHostToDevice, st)) != hipSuccess)
                return fail("bidomain upload");
            if (B.precond) {                         // x += M^{-1} V y
                k_combine<<<S.grid_c, BT, 0, st>>>(B.t, B.V, B.y, k, nc);
                S.prec(B.t, B.z);
                k_add<<<S.grid_c, BT, 0, st>>>(B.phi, B.z, nc);
            } else {
                k_update<<<S.grid_c, BT, 0, st>>>(B.phi, B.V, B.y, k, nc);
            }
            // y is pageable host memory: wait before it is rewritten
            if ((e = hipStreamSynchronize(st)) != hipSuccess) return fail("bidomain update");
        }
    }
    // zero volume-weighted mean
    S.dots(B.phi, D.vol, 1, h_norm + 1);
    k_shift<<<S.grid_c, BT, 0, st>>>(B.phi, h_norm + 1, 1.0 / B.total_vol, nc);
    if ((e = hipGetLastError()) != hipSuccess) return fail("bidomain kernels");
    B.last_iters = it;
    B.total_iters += it;
    B.last_relres = relres;
    return "";
}

}  // namespace ep
