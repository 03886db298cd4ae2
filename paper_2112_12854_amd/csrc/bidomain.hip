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
// solve gives the same bits on every run.  The (restart + 1) x restart
// Hessenberg least-squares problem (Givens rotations, the convergence test,
// back substitution) is advanced on the device by one-lane kernels, and the
// Arnoldi steps run in captured graphs of a few steps each whose kernels
// return at once after a device flag ends the cycle: the host reads the
// state back once per chunk and once per restart, never per Arnoldi step.
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
constexpr int NW = BT / 64;    // waves per block
constexpr int NQ = 8;          // dot products per pass of the reduction kernel
constexpr int G = kBidoBlocks; // blocks of the reduction kernels
constexpr int RMAX = kBidoMaxRestart;   // the longest restart the LDS staging holds

// node values by inverse-distance weights (sliced ELL, one lane per node)
// Kernels given a stop flag return at once while it is set (the Arnoldi
// steps enqueued past the end of a cycle).
__device__ __forceinline__ bool stopped(const int32_t *stop) { return stop && *stop; }

// (x scaled by *xs when xs is given)
__global__ void __launch_bounds__(BT) k_gather(const int64_t *__restrict__ off,
                                               const int32_t *__restrict__ cell,
                                               const double *__restrict__ w,
                                               const double *__restrict__ x,
                                               double *__restrict__ xn, int64_t nn,
                                               const int32_t *stop, const double *xs = nullptr) {
    if (stopped(stop)) return;
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
    xn[node] = xs ? *xs * ((a0 + a1) + (a2 + a3)) : (a0 + a1) + (a2 + a3);
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
                                             double *__restrict__ y, int64_t nc,
                                             const int32_t *stop) {
    if (stopped(stop)) return;
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
                                             double *__restrict__ part, const int32_t *stop) {
    if (stopped(stop)) return;
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
                                               double *__restrict__ out, const int32_t *stop) {
    if (stopped(stop)) return;
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
                                            const double *__restrict__ h, int cnt, int64_t n,
                                            const int32_t *stop) {
    if (stopped(stop)) return;
    const int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x;
    if (e >= n) return;
    double x = w[e];
    for (int q = 0; q < cnt; ++q) x -= h[q] * V[q * n + e];
    w[e] = x;
}

// x += sum_{q < *cnt} y_q s_q U_q (the count of the cycle's steps on the
// device; the basis vectors V_q = s_q U_q)
__global__ void __launch_bounds__(BT) k_update(double *__restrict__ x, const double *__restrict__ U,
                                               const double *__restrict__ y,
                                               const double *__restrict__ sc, const int32_t *cnt,
                                               int64_t n) {
    const int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x;
    const int k = *cnt;
    if (e >= n || k == 0) return;
    double acc = x[e];
    for (int q = 0; q < k; ++q) acc += y[q] * sc[q] * U[q * n + e];
    x[e] = acc;
}

// dst = a src, with a (a, or *ad when given) read on the device
__global__ void __launch_bounds__(BT) k_scale(double *__restrict__ dst, const double *__restrict__ src,
                                              double a, const double *ad, int64_t n,
                                              const int32_t *stop) {
    if (stopped(stop)) return;
    const int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x;
    if (e < n) dst[e] = (ad ? *ad : a) * src[e];
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
// rc[I] = sum of r over aggregate I (times *rs when given), in a fixed order.
// WAVE: one wave per aggregate (NW per block; small aggregates), lane l
// adding cells l, l + 64, ... of its list, then a butterfly; else one block
// per aggregate (large ones), thread t adding cells t, t + BT, ..., then a
// tree
template <bool WAVE>
__global__ void __launch_bounds__(BT) k_restrict(const double *__restrict__ r,
                                                 const int32_t *__restrict__ off,
                                                 const int32_t *__restrict__ cells,
                                                 double *__restrict__ rc, int32_t na, const int32_t *stop,
                                                 const double *rs) {
    if (stopped(stop)) return;
    if constexpr (WAVE) {
        const int lane = threadIdx.x & 63;
        const int32_t ag = blockIdx.x * NW + (threadIdx.x >> 6);
        if (ag >= na) return;
        double acc = 0.0;
        for (int32_t i = off[ag] + lane; i < off[ag + 1]; i += 64) acc += r[cells[i]];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane == 0) rc[ag] = rs ? *rs * acc : acc;
    } else {
        __shared__ double red[BT];
        double acc = 0.0;
        for (int32_t i = off[blockIdx.x] + threadIdx.x; i < off[blockIdx.x + 1]; i += BT) acc += r[cells[i]];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int s = BT / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) rc[blockIdx.x] = rs ? *rs * red[0] : red[0];
    }
}

// zc = A_c^{-1} rc (dense, row-major, FP32 entries, FP64 sums; one block per row)
__global__ void __launch_bounds__(BT) k_coarse(const float *__restrict__ cinv,
                                               const double *__restrict__ rc,
                                               double *__restrict__ zc, int32_t na,
                                               const int32_t *stop) {
    if (stopped(stop)) return;
    __shared__ double red[BT];
    const float *row = cinv + (int64_t)blockIdx.x * na;
    double acc = 0.0;
    for (int32_t j0 = threadIdx.x; j0 < na; j0 += 8 * BT) {   // 8 loads in flight per lane
        float c[8];
        double x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int32_t j = min(j0 + k * BT, na - 1);
            c[k] = row[j];
            x[k] = rc[j];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (j0 + k * BT < na) acc += (double)c[k] * x[k];
    }
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
                                               double *__restrict__ z, int64_t n,
                                               const int32_t *stop, const double *rs = nullptr) {
    if (stopped(stop)) return;
    const int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x;
    if (e < n) z[e] = omega * dinv[e] * (rs ? *rs * r[e] : r[e]) + zc[agg_of[e]];
}

// t = sum_{q < *cnt} y_q s_q U_q
__global__ void __launch_bounds__(BT) k_combine(double *__restrict__ t, const double *__restrict__ U,
                                                const double *__restrict__ y,
                                                const double *__restrict__ sc, const int32_t *cnt,
                                                int64_t n, const int32_t *stop) {
    if (stopped(stop)) return;
    const int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x;
    if (e >= n) return;
    const int k = *cnt;
    double acc = 0.0;
    for (int q = 0; q < k; ++q) acc += y[q] * sc[q] * U[q * n + e];
    t[e] = acc;
}

// x = 0 where *flag is set
__global__ void __launch_bounds__(BT) k_zero_if(double *__restrict__ x, const int32_t *flag, int64_t n) {
    if (!*flag) return;
    const int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x;
    if (e < n) x[e] = 0.0;
}

// x += z
__global__ void __launch_bounds__(BT) k_add(double *__restrict__ x, const double *__restrict__ z,
                                            int64_t n, const int32_t *stop) {
    if (stopped(stop)) return;
    const int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x;
    if (e < n) x[e] += z[e];
}

// ---- GMRES state on the device: one lane advances the Hessenberg
// least-squares problem exactly as the textbook method does on the host
struct GmCtl {
    double bnorm, beta, relres, pad0;  // |b|, |r| at the cycle start, |r|/|b|
    int32_t it, k, stop, done;         // Arnoldi steps so far, steps of this cycle, cycle over, solve over
    int32_t noupd, pad1[3];            // no update this cycle (k = 0)
};
static_assert(sizeof(GmCtl) == 64, "the control block takes the first 8 doubles");

// The basis is kept unnormalised: V_q = s_q U_q, s_q = 1 / |U_q|.
struct GmView {
    GmCtl *c;
    double *H, *cs, *sn, *g, *y, *s;   // H row-major (m + 1) x m; s: m + 1 scales
};
GmView gm_view(double *gm, int m) {
    GmView v;
    v.c = (GmCtl *)gm;
    v.H = gm + 8;
    v.cs = v.H + (size_t)(m + 1) * m;
    v.sn = v.cs + m;
    v.g = v.sn + m;
    v.y = v.g + (m + 1);
    v.s = v.y + m;
    return v;
}

__global__ void k_gm_init(GmCtl *c, const double *bb) {
    if (threadIdx.x) return;
    c->bnorm = sqrt(bb[0]);
    c->it = 0;
    c->k = 0;
    c->noupd = 1;
    c->relres = 0.0;
    c->done = c->stop = c->bnorm == 0.0;
}

// start of a restart cycle from the true residual's squared norm rr
__global__ void k_gm_start(GmView v, const double *rr, double tol, int32_t max_iter, int m) {
    if (threadIdx.x) return;
    GmCtl *c = v.c;
    c->k = 0;
    c->noupd = 1;
    if (c->done) { c->stop = 1; return; }
    c->beta = sqrt(rr[0]);
    c->relres = c->beta / c->bnorm;
    if (c->beta <= tol * c->bnorm || c->it >= max_iter) {
        c->done = c->stop = 1;
        return;
    }
    c->stop = 0;
    v.g[0] = c->beta;
    for (int i = 1; i <= m; ++i) v.g[i] = 0.0;
    v.s[0] = 1.0 / c->beta;
}

// Arnoldi step j (one lane, reading what the block staged in LDS): column j
// of H from the two Gram-Schmidt passes and the new norm (col: pass 1 +
// pass 2 for rows [0, j], cs/sn: the earlier rotations), the earlier
// rotations applied, a new one, the reduced right-hand side, the test, and
// the next basis scale, all written back to the device state
__device__ void gm_step(const GmView &v, double *col, const double *cs, const double *sn, double hn,
                        int j, int m, double tol, int32_t max_iter) {
    GmCtl *c = v.c;
    for (int i = 0; i < j; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = cs[i] * a + sn[i] * b;
        col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double hjj = col[j];
    const double den = hypot(hjj, hn);
    const double cj = den > 0.0 ? hjj / den : 1.0;
    const double sj = den > 0.0 ? hn / den : 0.0;
    col[j] = den;
    for (int i = 0; i <= j; ++i) v.H[(size_t)i * m + j] = col[i];
    v.H[(size_t)(j + 1) * m + j] = 0.0;
    v.cs[j] = cj;
    v.sn[j] = sj;
    const double gj = v.g[j];
    v.g[j + 1] = -sj * gj;
    v.g[j] = cj * gj;
    c->it += 1;
    c->k = j + 1;
    c->noupd = 0;
    if (fabs(sj * gj) <= tol * c->bnorm || hn == 0.0 || c->it >= max_iter || j == m - 1)
        c->stop = 1;
    else
        v.s[j + 1] = 1.0 / hn;
}

// R y = g for the cycle's k steps (back substitution), R and g staged in
// LDS by the block first
__global__ void __launch_bounds__(BT) k_gm_solve(GmView v, int m) {
    __shared__ double R[RMAX * RMAX], gl[RMAX], yl[RMAX];
    const int k = v.c->k;
    for (int t = threadIdx.x; t < k * k; t += blockDim.x) R[t] = v.H[(size_t)(t / k) * m + t % k];
    for (int t = threadIdx.x; t < k; t += blockDim.x) gl[t] = v.g[t];
    __syncthreads();
    if (threadIdx.x) return;
    for (int i = k - 1; i >= 0; --i) {
        double acc = gl[i];
        for (int l = i + 1; l < k; ++l) acc -= R[i * k + l] * yl[l];
        yl[i] = acc / R[i * k + i];
    }
    for (int i = 0; i < k; ++i) v.y[i] = yl[i];
}

// ---- Arnoldi-step kernels: the vector update of a step and the block
// partials of its dot products in one pass (one lane per cell), the rows
// then added by k_rows, one block per row, in a fixed order (so a solve
// still gives the same bits on every run).  A lane loads the basis values
// of R rows at once, so a pass waits for memory once per R rows: R = 32 on
// small grids, where the wait is what a pass costs, and R = 8 on large
// ones, where 32 rows at once would stream from 32 distant ranges of the
// basis (slower there than 8).
constexpr int RB = 32;         // the most rows per pass
static_assert(NW == 4, "the wave totals are added as (w0 + w1) + (w2 + w3)");

// a wave's 64 values added by a fixed butterfly (lane 0's result)
__device__ __forceinline__ double wave_sum(double a) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    return a;
}

// one exchange step of block_rows: rows [0, 2W) of a become rows [0, W),
// the lane keeping the half its bit O selects and adding the partner's
template <int W, int O, int R>
__device__ __forceinline__ void xstep(double (&a)[R], int lane) {
    const bool hi = (lane & O) != 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        const double keep = hi ? a[i + W] : a[i];
        const double give = hi ? a[i] : a[i + W];
        a[i] = keep + __shfl_xor(give, O, 64);
    }
}

// Block partials of R sums at once: a[q] holds the lane's term of row q.
// Within a wave, log2 R exchange steps (offsets 32, 16, ...) each hand half
// of the remaining rows to the partner lane and add, then the groups of
// 64 / R lanes that hold the same row add by a butterfly: lanes
// [r 64 / R, (r + 1) 64 / R) end with row r's wave total (one exchange per
// row and step instead of a butterfly per row).  The NW wave totals are
// added in a fixed order; row q < cnt of block b goes to
// part[q * gridDim.x + b].  Every addition has a fixed place, so the bits
// do not depend on timing.
template <int R>
__device__ __forceinline__ void block_rows(double (&a)[R], int cnt, double *part, double (*red)[RB]) {
    static_assert(R == 8 || R == 16 || R == 32, "R rows over 64 lanes");
    constexpr int G = 64 / R;  // lanes per row at the end
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    xstep<R / 2, 32>(a, lane);
    xstep<R / 4, 16>(a, lane);
    xstep<R / 8, 8>(a, lane);
    if constexpr (R >= 16) xstep<R / 16, 4>(a, lane);
    if constexpr (R >= 32) xstep<R / 32, 2>(a, lane);
    double t = a[0];
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if ((lane & (G - 1)) == 0) red[wave][lane / G] = t;
    __syncthreads();
    if ((int)threadIdx.x < cnt)
        part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
    __syncthreads();
}

// the lane's values of basis rows [q0, q0 + R) at element e (0 past cnt or
// n; cnt, n >= 1).  The loads themselves are unconditional, from the row and
// element clamped into range (rows past cnt re-read row cnt - 1 from the
// cache), so all R of them are in flight at once instead of one branch and
// one wait per row.
template <int R>
__device__ __forceinline__ void load_rows(double (&u)[R], const double *__restrict__ U, int q0,
                                          int cnt, int64_t n, int64_t e) {
    const int64_t ec = e < n ? e : n - 1;
    const double me = e < n ? 1.0 : 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q)
        u[q] = U[(int64_t)min(q0 + q, cnt - 1) * n + ec];
    // the mask as a product of finite values (every load read real data)
#pragma unroll
    for (int q = 0; q < R; ++q) u[q] *= q0 + q < cnt ? me : 0.0;
}

// the coefficients h_q s_q of rows [q0, q0 + R) (0 past cnt; sc null: h holds
// the products), loaded the same way
template <int R>
__device__ __forceinline__ void load_coef(double (&f)[R], const double *h, const double *__restrict__ sc,
                                          int q0, int cnt) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int qq = min(q0 + q, cnt - 1);
        const double x = sc ? h[qq] * sc[qq] : h[qq];
        f[q] = q0 + q < cnt ? x : 0.0;
    }
}

// Row sums of the previous pass inside its consumer (small grids, cnt <=
// RB rows): thread t adds partials t % 8, t % 8 + 8, ... of row t / 8, then
// the 8 lanes of the row add by a fixed butterfly, so every block holds the
// same bits; the sums times the scales (h_q) go, from block 0, to the global
// h read by the least-squares update, and h_q s_q to hs (LDS).
__device__ __forceinline__ void rows_in_block(const double *__restrict__ hp, int64_t np,
                                              const double *__restrict__ sc, int cnt,
                                              double *__restrict__ h, double *hs) {
    const int q = threadIdx.x >> 3, sg = threadIdx.x & 7;
    const double *p = hp + (int64_t)min(q, cnt - 1) * np;
    double acc = 0.0;
    for (int64_t i0 = sg; i0 < np; i0 += 64) {   // 8 loads in flight per lane
        double x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = p[min(i0 + 8 * k, np - 1)];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (i0 + 8 * k < np) acc += x[k];
    }
    if (q >= cnt) acc = 0.0;
    acc += __shfl_xor(acc, 4, 64);
    acc += __shfl_xor(acc, 2, 64);
    acc += __shfl_xor(acc, 1, 64);
    if (sg == 0 && q < cnt) {
        const double v = sc[q] * acc;
        hs[q] = v * sc[q];            // the coefficient h_q s_q of U_q
        if (blockIdx.x == 0) h[q] = v;
    }
    __syncthreads();
}

// w = A z (flux-sum form; node values zn already formed, z scaled by *zs
// when given), with the partials of <w, U_q>, q < cnt
template <int R>
__global__ void __launch_bounds__(BT) k_op_dots(const int32_t *__restrict__ cnode,
                                                const double *__restrict__ beta,
                                                const int32_t *__restrict__ cnbr,
                                                const double *__restrict__ bf,
                                                const double *__restrict__ z, const double *zs,
                                                const double *__restrict__ zn,
                                                double *__restrict__ w, const double *__restrict__ U,
                                                int cnt, int64_t nc, double *part, const int32_t *stop) {
    if (stopped(stop)) return;
    __shared__ double red[NW][RB];
    const int64_t c = blockIdx.x * (int64_t)BT + threadIdx.x;
    double y = 0.0;
    if (c < nc) {
        const double xc = z[c];
        double acc = 0.0;
#pragma unroll
        for (int s = 0; s < 8; ++s) acc += beta[tix(c, s, 8)] * zn[cnode[tix(c, s, 8)]];
        double two = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) two += bf[tix(c, q, 4)] * (z[cnbr[tix(c, q, 4)]] - xc);
        y = acc + (zs ? *zs : 1.0) * two;
        w[c] = y;
    }
    for (int q0 = 0; q0 < cnt; q0 += R) {
        double a[R];
        load_rows<R>(a, U, q0, cnt, nc, c);
#pragma unroll
        for (int q = 0; q < R; ++q) a[q] *= y;
        block_rows<R>(a, min(R, cnt - q0), part + (int64_t)q0 * gridDim.x, red);
    }
}

// w -= sum_{q < cnt} h_q V_q (in place), with the partials of <w, U_q>;
// with hp the h_q are first summed here from the previous pass's partials
template <int R>
__global__ void __launch_bounds__(BT) k_sub_dots(double *__restrict__ w, const double *__restrict__ U,
                                                 const double *__restrict__ sc,
                                                 double *__restrict__ h, int cnt, int64_t n,
                                                 double *part, const int32_t *stop,
                                                 const double *__restrict__ hp) {
    if (stopped(stop)) return;
    __shared__ double red[NW][RB];
    __shared__ double hs[RB];
    const double *hc = h, *scc = sc;
    if (hp) {
        rows_in_block(hp, gridDim.x, sc, cnt, h, hs);
        hc = hs;
        scc = nullptr;
    }
    const int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x;
    double x = e < n ? w[e] : 0.0;
    if (cnt <= R) {                // the rows stay in registers for the dots
        double u[R], f[R];
        load_coef<R>(f, hc, scc, 0, cnt);
        load_rows<R>(u, U, 0, cnt, n, e);
#pragma unroll
        for (int q = 0; q < R; ++q) x -= f[q] * u[q];
        if (e < n) w[e] = x;
#pragma unroll
        for (int q = 0; q < R; ++q) u[q] *= x;
        block_rows<R>(u, cnt, part, red);
        return;
    }
    for (int q0 = 0; q0 < cnt; q0 += R) {
        double u[R], f[R];
        load_coef<R>(f, hc, scc, q0, cnt);
        load_rows<R>(u, U, q0, cnt, n, e);
#pragma unroll
        for (int q = 0; q < R; ++q) x -= f[q] * u[q];
    }
    if (e < n) w[e] = x;
    for (int q0 = 0; q0 < cnt; q0 += R) {
        double u[R];
        load_rows<R>(u, U, q0, cnt, n, e);
#pragma unroll
        for (int q = 0; q < R; ++q) u[q] *= x;
        block_rows<R>(u, min(R, cnt - q0), part + (int64_t)q0 * gridDim.x, red);
    }
}

// U_{j+1} = w - sum_{q <= j} h_q V_q, with the partials of |U_{j+1}|^2;
// with hp the h_q are first summed here from the previous pass's partials
template <int R>
__global__ void __launch_bounds__(BT) k_sub_norm(const double *__restrict__ w, double *__restrict__ U,
                                                 const double *__restrict__ sc,
                                                 double *__restrict__ h, int j, int64_t n,
                                                 double *part, const int32_t *stop,
                                                 const double *__restrict__ hp) {
    if (stopped(stop)) return;
    __shared__ double red[NW];
    __shared__ double hs[RB];
    const double *hc = h, *scc = sc;
    if (hp) {
        rows_in_block(hp, gridDim.x, sc, j + 1, h, hs);
        hc = hs;
        scc = nullptr;
    }
    const int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x;
    double x = e < n ? w[e] : 0.0;
    for (int q0 = 0; q0 <= j; q0 += R) {
        double u[R], f[R];
        load_coef<R>(f, hc, scc, q0, j + 1);
        load_rows<R>(u, U, q0, j + 1, n, e);
#pragma unroll
        for (int q = 0; q < R; ++q) x -= f[q] * u[q];
    }
    if (e < n) U[(int64_t)(j + 1) * n + e] = x;
    const double t = wave_sum(e < n ? x * x : 0.0);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// out[q] = sc[q] * (sum of the np partials of row q) (or the sum); one block
// per row, lane t adding partials t, t + BT, ... in order, then a fixed tree
__global__ void __launch_bounds__(BT) k_rows(const double *__restrict__ part, int64_t np,
                                             const double *__restrict__ sc, double *__restrict__ out,
                                             const int32_t *stop) {
    if (stopped(stop)) return;
    __shared__ double red[BT];
    const double *p = part + (int64_t)blockIdx.x * np;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < np; i += BT) acc += p[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = BT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sc ? sc[blockIdx.x] * red[0] : red[0];
}

// |U_{j+1}|^2 from its partials, then the step's least-squares update (the
// column, the earlier rotations and the norm staged in LDS by all lanes)
__global__ void __launch_bounds__(BT) k_norm_step(const double *__restrict__ part, int64_t np, GmView v,
                                                  double *hd, int j, int m, double tol,
                                                  int32_t max_iter) {
    if (v.c->stop) return;
    __shared__ double red[BT];
    __shared__ double col[RMAX + 1], cs[RMAX], sn[RMAX];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < np; i += BT) acc += part[i];
    red[threadIdx.x] = acc;
    for (int i = threadIdx.x; i <= j; i += BT) col[i] = hd[i] + hd[m + 1 + i];
    for (int i = threadIdx.x; i < j; i += BT) {
        cs[i] = v.cs[i];
        sn[i] = v.sn[i];
    }
    __syncthreads();
    for (int s = BT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        hd[2 * (m + 1)] = red[0];
        gm_step(v, col, cs, sn, sqrt(red[0]), j, m, tol, max_iter);
    }
}

constexpr double kOmega = 0.7;   // Jacobi weight of the preconditioner
constexpr int kChunk = 4;        // Arnoldi steps per captured graph
constexpr int kFuseBlocks = 512; // grids up to this many blocks sum rows in the consumer

struct Solver {
    Inst &I;
    hipStream_t st;
    int64_t nc, nn;
    int grid_c, grid_n;

    // partial rows [row0, row0 + cnt) <- <w, V + q n>, then reduced into out[0..cnt)
    void dots(const double *w, const double *V, int cnt, double *out, const int32_t *stop = nullptr) {
        for (int q0 = 0; q0 < cnt; q0 += NQ) {
            const int k = std::min(NQ, cnt - q0);
            k_dots<<<G, BT, 0, st>>>(w, V + (int64_t)q0 * nc, k, nc, I.bd.part + (int64_t)q0 * G, stop);
        }
        k_reduce<<<cnt, BT, 0, st>>>(I.bd.part, out, stop);
    }
    // y = A x (elliptic operator, flux-sum form)
    void apply(const double *x, double *y, const int32_t *stop = nullptr) {
        const InstDesc &D = I.desc;
        k_gather<<<grid_n, BT, 0, st>>>(D.sell_off, D.sell_cell, (const double *)D.sell_w, x, I.bd.xn, nn,
                                        stop);
        k_flux<<<grid_c, BT, 0, st>>>(D.cnode, I.bd.ebeta, D.cnbr, I.bd.eb, x, I.bd.xn, nullptr, 1.0, y, nc,
                                      stop);
    }
    // rc = P^T r (times *rs): a wave per aggregate up to 128 cells per
    // aggregate on average, else a block
    void restrict_(const double *r, const double *rs, const int32_t *stop) {
        const Bido &B = I.bd;
        if (nc <= 128 * (int64_t)B.n_agg)
            k_restrict<true><<<(B.n_agg + NW - 1) / NW, BT, 0, st>>>(r, B.agg_off, B.agg_cells, B.rc, B.n_agg,
                                                                    stop, rs);
        else
            k_restrict<false><<<B.n_agg, BT, 0, st>>>(r, B.agg_off, B.agg_cells, B.rc, B.n_agg, stop, rs);
    }
    // z = M^{-1} r
    void prec(const double *r, double *z, const int32_t *stop = nullptr) {
        const Bido &B = I.bd;
        restrict_(r, nullptr, stop);
        k_coarse<<<B.n_agg, BT, 0, st>>>(B.cinv, B.rc, B.zc, B.n_agg, stop);
        k_smooth<<<grid_c, BT, 0, st>>>(r, B.dinv, B.agg_of, B.zc, kOmega, z, nc, stop);
    }
    // Arnoldi steps [j0, j1) of a cycle, each a no-op once the cycle is over:
    // 10 kernels each with the preconditioner (7 without); on small grids
    // the row sums of the two Gram-Schmidt passes happen inside their
    // consumers (8 kernels), the passes then alternating between two
    // partials buffers so that no block overwrites partials another still
    // reads
    void steps(int j0, int j1, const GmView &gv) {
        Bido &B = I.bd;
        const InstDesc &D = I.desc;
        const int m = B.restart;
        const int32_t *stop = &gv.c->stop;
        double *hd = B.h;
        const bool fuse = m + 1 <= RB && grid_c <= kFuseBlocks;
        double *pa = B.part;
        double *pb = fuse ? B.part + (size_t)(m + 1) * bido_part_cols(nc) : B.part;
        for (int j = j0; j < j1; ++j) {
            const double *uj = B.V + (int64_t)j * nc;
            const double *sj = gv.s + j;
            const double *z = uj, *zs = sj;
            if (B.precond) {                     // right preconditioning: z = M^{-1} V_j
                restrict_(uj, sj, stop);
                k_coarse<<<B.n_agg, BT, 0, st>>>(B.cinv, B.rc, B.zc, B.n_agg, stop);
                k_smooth<<<grid_c, BT, 0, st>>>(uj, B.dinv, B.agg_of, B.zc, kOmega, B.z, nc, stop, sj);
                z = B.z;
                zs = nullptr;
            }
            k_gather<<<grid_n, BT, 0, st>>>(D.sell_off, D.sell_cell, (const double *)D.sell_w, z, B.xn, nn,
                                            stop, zs);
            // w = A z with pass 1 of classical Gram-Schmidt, pass 2, then the
            // new vector, its norm and the least-squares update
            if (fuse) {
                k_op_dots<RB><<<grid_c, BT, 0, st>>>(D.cnode, B.ebeta, D.cnbr, B.eb, z, zs, B.xn, B.w, B.V,
                                                     j + 1, nc, pa, stop);
                k_sub_dots<RB><<<grid_c, BT, 0, st>>>(B.w, B.V, gv.s, hd, j + 1, nc, pb, stop, pa);
                k_sub_norm<RB><<<grid_c, BT, 0, st>>>(B.w, B.V, gv.s, hd + (m + 1), j, nc, pa, stop, pb);
            } else {
                k_op_dots<8><<<grid_c, BT, 0, st>>>(D.cnode, B.ebeta, D.cnbr, B.eb, z, zs, B.xn, B.w, B.V,
                                                    j + 1, nc, pa, stop);
                k_rows<<<j + 1, BT, 0, st>>>(pa, grid_c, gv.s, hd, stop);
                k_sub_dots<8><<<grid_c, BT, 0, st>>>(B.w, B.V, gv.s, hd, j + 1, nc, pb, stop, nullptr);
                k_rows<<<j + 1, BT, 0, st>>>(pb, grid_c, gv.s, hd + (m + 1), stop);
                k_sub_norm<8><<<grid_c, BT, 0, st>>>(B.w, B.V, gv.s, hd + (m + 1), j, nc, pa, stop, nullptr);
            }
            k_norm_step<<<1, BT, 0, st>>>(pa, grid_c, gv, hd, j, m, B.tol, B.max_iter);
        }
    }
    // the state's control block to the host
    hipError_t read(const GmView &gv) {
        hipError_t e = hipMemcpyAsync(I.bd.h_host, gv.c, sizeof(GmCtl), hipMemcpyDeviceToHost, st);
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
    const GmView gv = gm_view(B.gm, m);
    const double *v = (const double *)D.v[I.host_step & 1];
    double *const h_norm = B.h + 2 * (m + 1);   // |b|^2, |r|^2 (the steps' |w|^2 slot), then the mean
    const GmCtl *hc = (const GmCtl *)B.h_host;
    hipError_t e;
    auto fail = [&](const char *what) { return std::string(what) + ": " + hipGetErrorString(e); };


    // right-hand side: -chi Cm V_c L_i(v) = -(flux sums of v with M_i)
    k_gather<<<S.grid_n, BT, 0, st>>>(D.sell_off, D.sell_cell, (const double *)D.sell_w, v, B.xn, D.nn,
                                      nullptr);
    k_flux<<<S.grid_c, BT, 0, st>>>(D.cnode, (const double *)D.cbeta, D.cnbr, (const double *)D.cb, v,
                                    B.xn, D.vol, -B.chi_cm, B.b, nc, nullptr);
    S.dots(B.b, B.b, 1, h_norm);
    k_gm_init<<<1, 64, 0, st>>>(gv.c, h_norm);
    k_zero_if<<<S.grid_c, BT, 0, st>>>(B.phi, &gv.c->done, nc);   // b = 0: phi = 0
    {
        const int n_chunks = (m + kChunk - 1) / kChunk;
        if ((int)B.chunk_graphs.size() != n_chunks) B.chunk_graphs.assign(n_chunks, nullptr);
        // the previous solve's Arnoldi steps: the stop flag is read only from
        // two steps before that count on (every chunk in the first solve)
        const int64_t pred = B.last_iters;
        for (;;) {
            // the true residual r = b - A phi starts a cycle (or ends the
            // solve) as U_0, V_0 = r / |r|
            S.apply(B.phi, B.V);
            k_resid<<<S.grid_c, BT, 0, st>>>(B.V, B.b, nc);
            S.dots(B.V, B.V, 1, h_norm);
            k_gm_start<<<1, 64, 0, st>>>(gv, h_norm, B.tol, B.max_iter, m);
            if ((e = S.read(gv)) != hipSuccess) return fail("bidomain readback");
            if (hc->done) break;
            const int64_t it0 = hc->it;
            for (int q = 0; q < n_chunks; ++q) {
                if (!B.chunk_graphs[q]) {
                    hipGraph_t g = nullptr;
                    if ((e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                        return fail("bidomain capture");
                    S.steps(q * kChunk, std::min(m, (q + 1) * kChunk), gv);
                    if ((e = hipStreamEndCapture(st, &g)) != hipSuccess) return fail("bidomain capture");
                    e = hipGraphInstantiate(&B.chunk_graphs[q], g, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(g);
                    if (e != hipSuccess) { B.chunk_graphs[q] = nullptr; return fail("bidomain graph"); }
                }
                if ((e = hipGraphLaunch(B.chunk_graphs[q], st)) != hipSuccess) return fail("bidomain graph launch");
                if (q == n_chunks - 1 || it0 + std::min(m, (q + 1) * kChunk) + 2 < pred) continue;
                if ((e = S.read(gv)) != hipSuccess) return fail("bidomain readback");
                if (hc->stop) break;
            }
            k_gm_solve<<<1, BT, 0, st>>>(gv, m);
            if (B.precond) {                         // x += M^{-1} V y
                k_combine<<<S.grid_c, BT, 0, st>>>(B.t, B.V, gv.y, gv.s, &gv.c->k, nc, &gv.c->noupd);
                S.prec(B.t, B.z, &gv.c->noupd);
                k_add<<<S.grid_c, BT, 0, st>>>(B.phi, B.z, nc, &gv.c->noupd);
            } else {
                k_update<<<S.grid_c, BT, 0, st>>>(B.phi, B.V, gv.y, gv.s, &gv.c->k, nc);
            }
        }
    }
    // zero volume-weighted mean
    S.dots(B.phi, D.vol, 1, h_norm + 1);
    k_shift<<<S.grid_c, BT, 0, st>>>(B.phi, h_norm + 1, 1.0 / B.total_vol, nc);
    if ((e = hipGetLastError()) != hipSuccess) return fail("bidomain kernels");
    const int64_t it = hc->it;
    B.last_iters = it;
    B.total_iters += it;
    B.last_relres = hc->relres;
    return "";
}

}  // namespace ep
