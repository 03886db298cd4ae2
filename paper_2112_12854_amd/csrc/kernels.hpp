// Device kernels of the monodomain step, batched over simulation instances.
//
// Per step two kernels run over every live instance: the node gather (the
// inverse-distance node values of Sec. 3.2) and the fused cell kernel, which
// evaluates the face fluxes from the node values and neighbour potentials,
// the stimulus, the cell model, v^{n+1} = v^n + dt (L - I_ion - I_stim) and
// the activation / APD90 detection, all with level-n inputs.
//
// Work is described by tables in device memory: one descriptor per instance
// (its arrays, parameters and step counter) and lists of tiles of at most
// 256 cells or nodes, each inside one instance; one block per tile.  A
// captured graph is reused until the set of instances changes.  Every
// instance keeps its own step counter; v^n lives in buffer n & 1.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "cellmodels.hpp"

namespace epdev {

constexpr int MAX_STIM = 32;
constexpr int NG_MAX = 15;   // gate slots (CRN)
constexpr int NC_MAX = 6;    // FP64 slots (Stewart)
constexpr int TILE = 256;    // cells or nodes per tile (= block size)

// Per-cell slot arrays (stencil indices and coefficients, cell-model states)
// are tile-major: the S slots of the 256 cells of block b = c / 256 lie
// together, slot after slot ([block][slot][256]), so the accesses of a block
// to every slot of its cells stay inside one contiguous range.  An array
// holds S * ceil(n / 256) * 256 entries; the padding is never read.
constexpr int LB = 256;      // cells per layout block
__host__ __device__ constexpr size_t tiled_len(int64_t n, int S) {
    return (size_t)S * (size_t)((n + LB - 1) / LB) * LB;
}
__host__ __device__ constexpr size_t tix(int64_t c, int s, int S) {
    return ((size_t)(c / LB) * S + s) * LB + (size_t)(c % LB);
}

// Per-instance control block, device resident.
struct Ctrl {
    int64_t step;                 // index n of the next step of this instance
    int64_t target;               // the instance stops stepping at this index
    int32_t nan_flag;             // set when a non-finite v^{n+1} appears
    int32_t n_stim;
    int32_t pad[2];
    int64_t st_n0[MAX_STIM];      // first active step
    int64_t st_ndur[MAX_STIM];    // active steps per pulse
    int64_t st_nper[MAX_STIM];    // steps between pulses (0 = single pulse)
    int32_t st_count[MAX_STIM];   // pulses
    double st_amp[MAX_STIM];      // pA/pF
};

// A Purkinje-muscle junction.  fire_o / fire_a are the first steps of the
// pending stimuli of its muscle region / of its graph node.
struct Pmj {
    int64_t fire_o, fire_a;
    int64_t delay_o, delay_a, ndur;   // in steps
    double amp;
    double vprev;                     // junction node potential at the start of the step
    int32_t node, two_way;
    int32_t roff, rcnt;               // region: jcells[roff .. roff + rcnt)
    int32_t src_cell;                 // internal source cell, or -1 (graph node `node`)
    int32_t pad;
};
// cpmj_list entry: k pulses the cell with junction k's region pulse; k with
// kAntiFlag set with its two-way pulse (the cell is k's source)
constexpr int32_t kAntiFlag = 1 << 30;

// Everything a block needs to work on one instance (R = double or float
// arrays are passed as void and typed inside the kernels).
struct InstDesc {
    int64_t nc, nn;
    const int64_t *sell_off;
    const int32_t *sell_cell;
    const void *sell_w;
    const int32_t *cnode;         // tile-major, 8 slots (null with 16-bit ids)
    const void *cbeta;            // tile-major, 8 slots
    const int32_t *cnbr;          // tile-major, 4 slots (null with 16-bit ids)
    const void *cb;               // tile-major, 4 slots
    // 16-bit stencil ids (idx16 != 0): node id = nbase[c / 256] + cnode16,
    // neighbour id = cbase[c / 256] + cnbr16, when every 256-cell block's ids
    // span at most 65,535
    const uint16_t *cnode16;      // tile-major, 8 slots
    const uint16_t *cnbr16;       // tile-major, 4 slots
    const int32_t *nbase, *cbase; // [ceil(nc / 256)]
    int32_t idx16, pad16;
    void *vn;                     // [nn]
    void *v[2];                   // v^n in v[n & 1]
    void *gate;                   // tile-major, NG_MAX slots
    double *conc;                 // tile-major, NC_MAX slots
    const uint8_t *model;
    const uint32_t *smask;
    uint8_t *dstat;
    double *t_act, *t_rep;
    void *vmax;
    const void *vrest;
    const double *vol;
    double *part;                 // one partial sum per wave of 64 cells (zero-padded to 4)
    double *trace;                // vbar samples
    Ctrl *ctrl;
    double dt, thr, repol, inv_total_vol;
    GScale gs;
    int64_t trace_cap;
    int32_t trace_every;
    int32_t n_waves;              // wave partials: ceil(len / 64) per class range
    // bidomain: the extracellular potential phi_e^n (FP64; null otherwise);
    // the flux of the time step is then that of v + phi_e
    const double *phi;
    // junction stimuli of the muscle (null without a Purkinje graph)
    const int32_t *cpmj;          // [nc]: -1 or start of a -1-terminated list
    const int32_t *cpmj_list;
    const Pmj *pmj;
    // Adams-Bashforth 2 for the non-gating states (null: forward Euler):
    // the previous step's rate of v (R, [nc]) and of the model's non-gating
    // states (FP64, tile-major, NC_MAX slots)
    void *hv;
    double *hc;
    // a 2D medium with a time step of its own: the potentials between its
    // substeps (R, indexed by internal cell; only its cells are valid) and
    // its substep dt / n_sub
    void *w[2];
    double dt2;
};

// The potentials a substep reads and writes.  Substep q of m (m = 1: the
// plain step) reads v^n (q = 0) or w[(q - 1) & 1] and writes v^{n+1}
// (q = m - 1) or w[q & 1]; the step's level-n buffers stay untouched until
// its last substep, so junction events still see v^n.
struct Sub {
    const void *vin;
    void *vout;
    double dt;                    // dt / m
    int64_t t;                    // n m + q: start of the substep in units of dt / m
    bool first;                   // the instance's first update (n = 0, q = 0)
    bool last;                    // q = m - 1
};
__device__ __forceinline__ Sub substep(const InstDesc &D, int64_t n, int32_t q, int32_t m) {
    Sub sb;
    sb.vin = q == 0 ? D.v[n & 1] : D.w[(q - 1) & 1];
    sb.vout = q == m - 1 ? D.v[(n + 1) & 1] : D.w[q & 1];
    sb.dt = m == 1 ? D.dt : D.dt2;
    sb.t = n * m + q;
    sb.first = n == 0 && q == 0;
    sb.last = q == m - 1;
    return sb;
}

// A Purkinje graph (vertex-centred finite volumes on a 1D graph) coupled to
// an instance: CSR operator, states, detection and junctions.
struct PurkDesc {
    int64_t np;
    int32_t n_sub, n_pmj, model, pad;
    const int32_t *off, *nbr;
    const void *g;                // [off[np]] coefficients of (v_j - v_i)
    void *pv[2];                  // substep q reads pv[q & 1], writes pv[(q+1) & 1]
    void *gate;                   // tile-major over nodes, NG_MAX slots
    double *conc;                 // tile-major over nodes, NC_MAX slots
    const uint32_t *pmask;        // graph stimuli holding the node
    uint8_t *pstat;
    double *pt_act;
    const int32_t *npmj;          // [np]: -1 or start of a list of two-way junctions
    const int32_t *npmj_list;
    Pmj *pmj;
    const int32_t *jcells;
    const void *tv[2];            // the instance's tissue potential buffers
    Ctrl *ctrl;
    double dtp, thr;
    GScale gs;
    void *hv;                     // Adams-Bashforth 2 history, as in InstDesc
    double *hc;
};

// A tile carries a copy of its instance's descriptor, so a block reaches
// all it needs with one scalar load chain.
struct Tile {
    InstDesc d;
    int64_t begin;                // first cell / node of the tile
    int32_t count;                // cells / nodes in the tile (<= TILE)
    int32_t local;                // tile index inside its instance
    int32_t sub_m;                // substeps per step of the tile's medium (1: none)
    int32_t wave0;                // cell tiles: index of the wave partial of its first cell
};

// The launch grids always equal the tile counts (graphs are re-captured when
// the counts change), so kernels index the tables without a bound check.
struct PTile {
    PurkDesc p;
    int64_t begin;
    int32_t count, local;
};

struct Tables {
    const InstDesc *desc;         // one per instance (for the step counters)
    const Tile *cell_tiles;
    const Tile *node_tiles;
    const PTile *purk_tiles;
    const PurkDesc *purk;         // one per instance with a Purkinje graph
    const int32_t *counts;        // [0] cell tiles, [1] node tiles, [2] instances,
                                  // [3] graph tiles, [4] graphs
};

// Blocks are dealt round-robin to the 8 XCDs; remap block b so that each XCD
// works on one contiguous range of tiles and its L2 holds the neighbour data
// of that range.  A bijection of [0, nb).
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
    const int64_t x = b & 7, i = b >> 3;
    const int64_t q = nb >> 3, r = nb & 7;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Remap 2: the contiguous ranges of remap 1 taken over chunks of tiles
// instead of tiles: the first 8 R whole chunks (R per XCD, kXcdChunks = 8 R
// chunks of nb / (8 R) tiles) are transposed so that XCD x works on chunks
// x, x + 8, x + 16, ... spread over the whole tile range (the work of a
// region that costs more per cell is shared by all XCDs), each chunk still
// a contiguous range whose neighbour data stays in that XCD's L2; tiles
// past the whole chunks keep their place.  A bijection of [0, nb).
constexpr int kXcdRows = 4;
__device__ __forceinline__ int64_t chunk_tile(int64_t t, int64_t nb) {
    const int64_t K = nb / (8 * kXcdRows);          // tiles per chunk
    if (K == 0 || t >= 8 * kXcdRows * K) return t;
    const int64_t c = t / K, o = t - c * K;
    return ((c % kXcdRows) * 8 + c / kXcdRows) * K + o;
}

__device__ __forceinline__ int64_t my_tile(int remap) {
    if (remap == 0) return (int64_t)blockIdx.x;
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x);
    return remap == 1 ? t : chunk_tile(t, gridDim.x);
}

__device__ __forceinline__ bool stepping(const Ctrl *ctrl, int32_t off, int64_t &n) {
    n = ctrl->step + off;
    return n < ctrl->target;
}

// Trace of vbar.  On a sample step every wave of cells (64 consecutive
// cells of one class range) stores the sum of V_c v_c over its cells,
// reduced across the wave by a fixed butterfly (lane 0's result); the first
// node tile of the next step adds the wave partials (complete by then: the
// kernels are stream ordered), so no tile waits on another and the order of
// the additions is fixed: lane t adds the groups of four partials t,
// t + 256, ..., each as (p0 + p1) + (p2 + p3), then a fixed tree.  Neither
// the partials nor their sum depend on the cell tile shape.  A sample taken
// by the last step issued is reduced the same way on the host.
__device__ __forceinline__ void wave_partial(const InstDesc &D, int64_t idx, double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63) == 0) D.part[idx] = x;
}

__device__ __forceinline__ void reduce_trace(const InstDesc &D, int64_t idx, double *red) {
    double acc = 0.0;
    const int ng = (D.n_waves + 3) / 4;
    for (int g = threadIdx.x; g < ng; g += TILE) {
        const double *p = D.part + 4 * (int64_t)g;
        acc += (p[0] + p[1]) + (p[2] + p[3]);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = TILE / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && idx < D.trace_cap) D.trace[idx] = red[0] * D.inv_total_vol;
}

// Bit i set when stimulus i is on during step n (integer step windows).
__device__ __forceinline__ uint32_t active_stimuli(const Ctrl *ctrl, int64_t n) {
    uint32_t active = 0;
    const int ns = ctrl->n_stim;
    for (int i = 0; i < ns; ++i) {
        const int64_t k = n - ctrl->st_n0[i];
        const int64_t per = ctrl->st_nper[i];
        const bool on = k >= 0 && (per <= 0 ? k < ctrl->st_ndur[i]
                                            : (k / per) < ctrl->st_count[i] &&
                                                  (k % per) < ctrl->st_ndur[i]);
        active |= (on ? 1u : 0u) << i;
    }
    return active;
}

// ------------------------------------------------------------ node gather
// Inverse-distance node value v_n = sum_k w_nk v_k of node `node` from the
// cell potentials v (sliced ELL: 64 nodes per slice, entry j of a node at
// slice offset + j * 64).  Four independent gathers in flight per lane and
// a fixed summation order, so every caller gets the same bits.
template <typename R>
__device__ __forceinline__ R node_value(const InstDesc &D, int64_t node, const R *__restrict__ v) {
    const R *__restrict__ w8 = (const R *)D.sell_w;
    const int32_t *__restrict__ cell = D.sell_cell;
    const int64_t e0 = D.sell_off[node >> 6] + (node & 63), e1 = D.sell_off[(node >> 6) + 1];
    R a0 = R(0), a1 = R(0), a2 = R(0), a3 = R(0);
    int64_t e = e0;
    for (; e + 192 < e1; e += 256) {
        const int32_t c0 = cell[e], c1 = cell[e + 64], c2 = cell[e + 128], c3 = cell[e + 192];
        const R x0 = w8[e], x1 = w8[e + 64], x2 = w8[e + 128], x3 = w8[e + 192];
        a0 += x0 * v[c0];
        a1 += x1 * v[c1];
        a2 += x2 * v[c2];
        a3 += x3 * v[c3];
    }
    for (; e < e1; e += 64) a0 += w8[e] * v[cell[e]];
    return (a0 + a1) + (a2 + a3);
}

// BIDO: node values of v + phi_e (bidomain time step, FP64).
// sub < 0: the step's node values (every tile of the launch steps once);
// sub = q >= 0: those of substep q of a medium with substeps (tiles whose
// medium takes q or fewer substeps sit it out).
template <typename R, bool BIDO = false>
__global__ void __launch_bounds__(TILE) k_node_gather(Tables tb, int32_t step_off, int remap,
                                                      int32_t sub) {
    const Tile &T = tb.node_tiles[my_tile(remap)];
    const InstDesc &D = T.d;
    int64_t n;
    if (!stepping(D.ctrl, step_off, n)) return;
    if (sub >= T.sub_m) return;
    if (T.local == 0 && sub <= 0 && D.trace_every > 0 && n > 0 && n % D.trace_every == 0) {
        __shared__ double red[TILE];
        reduce_trace(D, n / D.trace_every, red);
    }
    if ((int32_t)threadIdx.x >= T.count) return;
    const int64_t node = T.begin + threadIdx.x;
    const R *__restrict__ v = (const R *)(sub <= 0 ? D.v[n & 1] : D.w[(sub - 1) & 1]);
    if constexpr (!BIDO) {
        ((R *)D.vn)[node] = node_value<R>(D, node, v);
    } else {
        // as node_value, of v + phi_e
        const R *__restrict__ w8 = (const R *)D.sell_w;
        const int32_t *__restrict__ cell = D.sell_cell;
        const double *__restrict__ ph = D.phi;
        const int64_t e0 = D.sell_off[node >> 6] + (node & 63), e1 = D.sell_off[(node >> 6) + 1];
        R a0 = R(0), a1 = R(0), a2 = R(0), a3 = R(0);
        int64_t e = e0;
        for (; e + 192 < e1; e += 256) {
            const int32_t c0 = cell[e], c1 = cell[e + 64], c2 = cell[e + 128], c3 = cell[e + 192];
            const R x0 = w8[e], x1 = w8[e + 64], x2 = w8[e + 128], x3 = w8[e + 192];
            a0 += x0 * (v[c0] + R(ph[c0]));
            a1 += x1 * (v[c1] + R(ph[c1]));
            a2 += x2 * (v[c2] + R(ph[c2]));
            a3 += x3 * (v[c3] + R(ph[c3]));
        }
        for (; e < e1; e += 64) a0 += w8[e] * (v[cell[e]] + R(ph[cell[e]]));
        ((R *)D.vn)[node] = (a0 + a1) + (a2 + a3);
    }
}

// ------------------------------------------------------------- cell step
// Per-cell arrays are addressed as a uniform base plus a 32-bit byte offset
// (scalar-base + vector-offset loads: one offset register serves every array
// instead of a 64-bit address pair per array).  Instances stay below 2^29
// cells, so the byte offsets of 8-byte elements fit.
template <typename T>
__device__ __forceinline__ T *slot(T *p, int s, int64_t n) { return p + (int64_t)s * n; }
template <typename T>
__device__ __forceinline__ T &at(T *p, uint32_t c) {
    return *(T *)((char *)p + c * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ const T &at(const T *p, uint32_t c) {
    return *(const T *)((const char *)p + c * (uint32_t)sizeof(T));
}

// Tile-major slot arrays go through buffer resources: one resource and one
// lane offset serve every slot of an array, the slot is a constant scalar
// offset.  Offsets are 32-bit, so an instance holds fewer than 2^25 cells
// (checked on the host).
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, -1, 0x00020000);
}
// Cache policy of buffer accesses: kStream marks data touched once per step
// (stencil coefficients, cell-model states) as non-temporal, so that it does
// not evict the node values and neighbour potentials the gathers reuse.
constexpr int kCached = 0, kStream = 2;
template <typename T> struct BufIO;
template <> struct BufIO<float> {
    template <int P>
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, P));
    }
    template <int P>
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, float x, uint32_t v, uint32_t s) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, v, s, P);
    }
};
template <> struct BufIO<uint16_t> {
    template <int P>
    static __device__ __forceinline__ uint16_t ld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
        return __builtin_amdgcn_raw_buffer_load_b16(r, v, s, P);
    }
};
template <> struct BufIO<int32_t> {
    template <int P>
    static __device__ __forceinline__ int32_t ld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
        return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(r, v, s, P);
    }
};
template <> struct BufIO<double> {
    template <int P>
    static __device__ __forceinline__ double ld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, P));
    }
    template <int P>
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, double x, uint32_t v, uint32_t s) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, x), r, v, s, P);
    }
};
// byte offset of slot 0 of element c in a tile-major array of S slots
template <typename T, int S>
__device__ __forceinline__ uint32_t lane_off(uint32_t c) {
    return ((c >> 8) * (uint32_t)(S * LB) + (c & (uint32_t)(LB - 1))) * (uint32_t)sizeof(T);
}
// slot s of element c of a tile-major array of S slots
template <typename T, int S, int P = kStream>
__device__ __forceinline__ T sld(__amdgpu_buffer_rsrc_t r, int s, uint32_t c) {
    return BufIO<T>::template ld<P>(r, lane_off<T, S>(c), (uint32_t)(s * LB * (int)sizeof(T)));
}
template <typename T, int S, int P = kStream>
__device__ __forceinline__ void sst(__amdgpu_buffer_rsrc_t r, int s, uint32_t c, T x) {
    BufIO<T>::template st<P>(r, x, lane_off<T, S>(c), (uint32_t)(s * LB * (int)sizeof(T)));
}

// One cell-model update of cell c of a tile-major state set: gates by
// Rush-Larsen, FP64 concentrations by forward Euler, all from level-n values.
// Returns I_ion at level n (0 for passive cells).
// MSET: bit 0 TP06 (any layer), 1 CRN, 2 Stewart, 3 passive.
// One cell model over one step: load its gates and non-gating states (and,
// with AB2, the previous rates of the latter), step, store.
template <typename R, int NG, int NC, bool AB2, typename F>
__device__ __forceinline__ R model_io(__amdgpu_buffer_rsrc_t rgate, __amdgpu_buffer_rsrc_t rconc,
                                      __amdgpu_buffer_rsrc_t rhist, uint32_t c, bool first,
                                      F &&fn) {
    R g[NG_MAX];
    double cc[NC_MAX], hh[NC_MAX];
#pragma unroll
    for (int s = 0; s < NG; ++s) g[s] = sld<R, NG_MAX>(rgate, s, c);
#pragma unroll
    for (int s = 0; s < NC; ++s) cc[s] = sld<double, NC_MAX>(rconc, s, c);
    R iion;
    if constexpr (AB2) {
        if (!first) {
#pragma unroll
            for (int s = 0; s < NC; ++s) hh[s] = sld<double, NC_MAX>(rhist, s, c);
        }
        iion = fn(g, cc, AdamsBashforth2{hh, first});
#pragma unroll
        for (int s = 0; s < NC; ++s) sst<double, NC_MAX>(rhist, s, c, hh[s]);
    } else {
        iion = fn(g, cc, FwdEuler{});
    }
#pragma unroll
    for (int s = 0; s < NG; ++s) sst<R, NG_MAX>(rgate, s, c, g[s]);
#pragma unroll
    for (int s = 0; s < NC; ++s) sst<double, NC_MAX>(rconc, s, c, cc[s]);
    return iion;
}

// Time schemes: 0 Rush-Larsen + forward Euler (the paper's), 1 Rush-Larsen
// + Adams-Bashforth 2 for the non-gating states, 2 as 1 with the gates'
// rates at midpoint predictions (second order overall).
template <typename R, int MSET, int SCH = 0>
__device__ __forceinline__ R ionic(int md, R v, __amdgpu_buffer_rsrc_t rgate,
                                   __amdgpu_buffer_rsrc_t rconc, uint32_t c, R dt,
                                   double dtd, R istim, const GScale &gs,
                                   __amdgpu_buffer_rsrc_t rhist = rsrc(nullptr),
                                   bool first = false, R lmi = R(0)) {
    constexpr bool HIST = SCH >= 1, MID = SCH == 2;
    R iion = R(0);
    if ((MSET & 1) && md <= 2) {
        iion = model_io<R, tp06::NG, tp06::NC, HIST>(
            rgate, rconc, rhist, c, first, [&](R *g, double *cc, const auto &e) {
                return tp06::step<R, MID>(md, v, g, cc, dt, dtd, istim, gs, e, lmi);
            });
    } else if ((MSET & 2) && md == 3) {
        iion = model_io<R, crn::NG, crn::NC, HIST>(
            rgate, rconc, rhist, c, first, [&](R *g, double *cc, const auto &e) {
                return crn::step<R, MID>(v, g, cc, dt, dtd, gs, e, lmi);
            });
    } else if ((MSET & 4) && md == 4) {
        iion = model_io<R, stewart::NG, stewart::NC, HIST>(
            rgate, rconc, rhist, c, first, [&](R *g, double *cc, const auto &e) {
                return stewart::step<R, MID>(v, g, cc, dt, dtd, istim, gs, e, lmi);
            });
    }
    return iion;
}

// v^{n+1} from v^n and its rate: forward Euler, or Adams-Bashforth 2 with
// the previous rate in hv[i] (forward Euler on the first step).
template <typename R, bool AB2>
__device__ __forceinline__ R v_update(R v, R dt, R F, void *hv, uint32_t i, bool first) {
    if constexpr (AB2) {
        R *h = (R *)hv;
        const R p = first ? F : h[i];
        h[i] = F;
        return v + dt * (R(1.5) * F - R(0.5) * p);
    } else {
        return v + dt * F;
    }
}

// Face-flux sum of cell c in mV/ms: L_c = sum_f F_f / (chi Cm V_c), from
// the per-cell fused coefficients (gradient of the node values through the
// eight node weights, two-point terms along the four neighbours), the node
// values vn and the cell potentials vin; v = vin[c].  BIDO: the flux of
// v + phi_e (vn then holds node values of v + phi_e).
template <typename R, bool BIDO>
__device__ __forceinline__ R flux_sum(const InstDesc &D, uint32_t c, const R *__restrict__ vin,
                                      const R *__restrict__ vn, R v) {
    const __amdgpu_buffer_rsrc_t rbeta = rsrc(D.cbeta), rb = rsrc(D.cb);
    R L = R(0);
    auto stencil = [&](auto node_id, auto nbr_id) {
#pragma unroll
        for (int s = 0; s < 8; ++s) L += sld<R, 8>(rbeta, s, c) * at(vn, node_id(s));
        if constexpr (BIDO) {
            // the flux of u = v + phi_e (node values above are those of u)
            const R uc = v + R(at(D.phi, c));
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const uint32_t k = nbr_id(f);
                L += sld<R, 4>(rb, f, c) * ((at(vin, k) + R(at(D.phi, k))) - uc);
            }
        } else {
#pragma unroll
            for (int f = 0; f < 4; ++f) L += sld<R, 4>(rb, f, c) * (at(vin, nbr_id(f)) - v);
        }
    };
    if (D.idx16) {
        const __amdgpu_buffer_rsrc_t rn16 = rsrc(D.cnode16), rf16 = rsrc(D.cnbr16);
        const uint32_t nb = (uint32_t)at(D.nbase, c >> 8), fb = (uint32_t)at(D.cbase, c >> 8);
        stencil([&](int s) { return nb + (uint32_t)sld<uint16_t, 8>(rn16, s, c); },
                [&](int f) { return fb + (uint32_t)sld<uint16_t, 4>(rf16, f, c); });
    } else {
        const __amdgpu_buffer_rsrc_t rnode = rsrc(D.cnode), rnbr = rsrc(D.cnbr);
        stencil([&](int s) { return (uint32_t)sld<int32_t, 8>(rnode, s, c); },
                [&](int f) { return (uint32_t)sld<int32_t, 4>(rnbr, f, c); });
    }
    return L;
}

template <typename R, int MSET, bool BIDO, int SCH>
__device__ __forceinline__ void cell_step(const InstDesc &D, uint32_t c, int64_t n,
                                          uint32_t active, bool sample, double &vol_v,
                                          const Sub &sb) {
    constexpr bool AB2 = SCH >= 1;
    const R *__restrict__ vin = (const R *)sb.vin;
    R *__restrict__ vout = (R *)sb.vout;
    const R *__restrict__ vn = (const R *)D.vn;

    // ---- diffusion: fused node-coefficient stencil plus two-point terms
    const R v = at(vin, c);
    const R L = flux_sum<R, BIDO>(D, c, vin, vn, v);

    // ---- stimulus: protocol pulses, then junction pulses (junction order)
    R istim = R(0);
    if (active) {
        uint32_t m = at(D.smask, c) & active;
        while (m) {
            const int i = __ffs(m) - 1;
            istim += R(D.ctrl->st_amp[i]);
            m &= m - 1;
        }
    }
    if (D.cpmj) {
        int32_t q = at(D.cpmj, c);
        if (q >= 0)
            for (int32_t k; (k = D.cpmj_list[q]) >= 0; ++q) {
                const Pmj &J = D.pmj[k & (kAntiFlag - 1)];
                const int64_t f = (k & kAntiFlag) ? J.fire_a : J.fire_o;
                if (n >= f && n < f + J.ndur) istim += R(J.amp);
            }
    }

    // ---- cell model
    const int md = (MSET == 8) ? 5 : __builtin_nontemporal_load(&D.model[c]);   // TP06 layer or model id
    const R dt = R(sb.dt);
    R iion;
    if constexpr (AB2)
        iion = ionic<R, MSET, SCH>(md, v, rsrc(D.gate), rsrc(D.conc), c, dt, sb.dt, istim,
                                   D.gs, rsrc(D.hc), sb.first, L - istim);
    else
        iion = ionic<R, MSET>(md, v, rsrc(D.gate), rsrc(D.conc), c, dt, sb.dt, istim, D.gs);

    // ---- explicit update of v
    const R vnew = v_update<R, AB2>(v, dt, L - iion - istim, D.hv, c, sb.first);
    at(vout, c) = vnew;
    if (!(fabs(vnew) < R(1e30))) atomicOr(&D.ctrl->nan_flag, 1);
    if (sample) vol_v = at(D.vol, c) * double(vnew);

    // ---- activation time and APD90 (streamed, like the states: the node
    // values and potentials the gathers reuse keep the cache)
    const uint8_t st = __builtin_nontemporal_load(&D.dstat[c]);
    if (st == 0) {
        const R thr = R(D.thr);
        if (v <= thr && vnew > thr) {
            __builtin_nontemporal_store((double(sb.t) + double((thr - v) / (vnew - v))) * sb.dt, &D.t_act[c]);
            __builtin_nontemporal_store(vnew, &((R *)D.vmax)[c]);
            __builtin_nontemporal_store((uint8_t)1, &D.dstat[c]);
        }
    } else if (st == 1) {
        R vm = __builtin_nontemporal_load(&((const R *)D.vmax)[c]);
        if (vnew > vm) {
            vm = vnew;
            __builtin_nontemporal_store(vm, &((R *)D.vmax)[c]);
        }
        const R v90 = vm - R(D.repol) * (vm - __builtin_nontemporal_load(&((const R *)D.vrest)[c]));
        if (v >= v90 && vnew < v90) {
            __builtin_nontemporal_store((double(sb.t) + double((v - v90) / (v - vnew))) * sb.dt, &D.t_rep[c]);
            __builtin_nontemporal_store((uint8_t)2, &D.dstat[c]);
        }
    }
}

// One launch per model class: the host passes tb.cell_tiles pointing at the
// first tile of the class in the class-ordered tile list.
// sub < 0: one step of every tile of the launch; sub = q >= 0: substep q of
// the tiles of a medium with substeps (as in k_node_gather).  A cell tile
// holds up to blockDim.x cells, one per lane (64, 128 or 256: the tile shape
// is a launch choice, and no result depends on it).
template <typename R, int MSET, bool BIDO = false, int SCH = 0>
__global__ void __launch_bounds__(TILE) k_cell(Tables tb, int32_t step_off, int remap,
                                               int32_t sub) {
    const Tile &T = tb.cell_tiles[my_tile(remap)];
    const InstDesc &D = T.d;
    int64_t n;
    if (!stepping(D.ctrl, step_off, n)) return;
    if (sub >= T.sub_m) return;
    const Sub sb = substep(D, n, sub < 0 ? 0 : sub, sub < 0 ? 1 : T.sub_m);
    const uint32_t active = active_stimuli(D.ctrl, n);
    const bool sample = sb.last && D.trace_every > 0 && (n + 1) % D.trace_every == 0;
    const int32_t i = (int32_t)threadIdx.x;
    double x = 0.0;
    if (i < T.count)
        cell_step<R, MSET, BIDO, SCH>(D, (uint32_t)(T.begin + i), n, active, sample, x, sb);
    if (sample && (i & ~63) < T.count) wave_partial(D, T.wave0 + (i >> 6), x);
}

// ------------------------------------------------------- Purkinje graph
// Substep `sub` of step n of every graph: explicit update of node i with the
// graph flux, the stimuli of the graph and of its two-way junctions, and the
// node's cell model over dt / n_sub; first upward threshold crossing.
template <typename R, int SCH = 0>
__global__ void __launch_bounds__(TILE) k_purkinje(Tables tb, int32_t step_off, int32_t sub) {
    constexpr bool AB2 = SCH >= 1;
    const PTile &T = tb.purk_tiles[blockIdx.x];
    const PurkDesc &P = T.p;
    int64_t n;
    if (!stepping(P.ctrl, step_off, n) || sub >= P.n_sub) return;
    const uint32_t active = active_stimuli(P.ctrl, n);
    if ((int32_t)threadIdx.x >= T.count) return;
    const uint32_t i = (uint32_t)(T.begin + threadIdx.x);
    const int64_t q = n * P.n_sub + sub;
    const R *__restrict__ vin = (const R *)P.pv[q & 1];
    R *__restrict__ vout = (R *)P.pv[(q + 1) & 1];
    const R *__restrict__ g = (const R *)P.g;
    const R v = vin[i];
    R L = R(0);
    for (int32_t e = P.off[i]; e < P.off[i + 1]; ++e) L += g[e] * (vin[P.nbr[e]] - v);
    R istim = R(0);
    uint32_t m = P.pmask[i] & active;
    while (m) {
        const int k = __ffs(m) - 1;
        istim += R(P.ctrl->st_amp[k]);
        m &= m - 1;
    }
    int32_t l = P.npmj[i];
    if (l >= 0)
        for (int32_t k; (k = P.npmj_list[l]) >= 0; ++l) {
            const Pmj &J = P.pmj[k];
            if (n >= J.fire_a && n < J.fire_a + J.ndur) istim += R(J.amp);
        }
    const R dt = R(P.dtp);
    R iion;
    if constexpr (AB2)
        iion = ionic<R, 15, SCH>(P.model, v, rsrc(P.gate), rsrc(P.conc), i, dt, P.dtp,
                                 istim, P.gs, rsrc(P.hc), q == 0, L - istim);
    else
        iion = ionic<R, 15>(P.model, v, rsrc(P.gate), rsrc(P.conc), i, dt, P.dtp, istim,
                            P.gs);
    const R vnew = v_update<R, AB2>(v, dt, L - iion - istim, P.hv, i, q == 0);
    vout[i] = vnew;
    if (!(fabs(vnew) < R(1e30))) atomicOr(&P.ctrl->nan_flag, 1);
    const R thr = R(P.thr);
    if (P.pstat[i] == 0 && v <= thr && vnew > thr) {
        P.pt_act[i] = (double(q) + double((thr - v) / (vnew - v))) * P.dtp;
        P.pstat[i] = 1;
    }
}

// Junction events of step n, after the graph substeps: an upward crossing at
// the junction node schedules the muscle pulse, an upward crossing of the
// region's mean potential (two-way junctions) schedules the node pulse.
// One block per graph; one thread per junction.
template <typename R>
__global__ void __launch_bounds__(TILE) k_junctions(Tables tb, int32_t step_off) {
    const PurkDesc &P = tb.purk[blockIdx.x];
    int64_t n;
    if (!stepping(P.ctrl, step_off, n)) return;
    const R *vp = (const R *)P.pv[((n + 1) * P.n_sub) & 1];
    const R *v0 = (const R *)P.tv[n & 1];
    const R *v1 = (const R *)P.tv[(n + 1) & 1];
    const R thr = R(P.thr);
    for (int32_t k = threadIdx.x; k < P.n_pmj; k += blockDim.x) {
        Pmj &J = P.pmj[k];
        // source: a graph node (its potential at the start of the step is
        // kept in vprev) or a cell (the tissue's v^n and v^{n+1})
        R a, b;
        if (J.src_cell >= 0) {
            a = v0[J.src_cell];
            b = v1[J.src_cell];
        } else {
            a = R(J.vprev);
            b = vp[J.node];
            J.vprev = double(b);
        }
        if (a <= thr && b > thr) J.fire_o = n + 1 + J.delay_o;
        if (J.two_way) {
            double m0 = 0.0, m1 = 0.0;
            for (int32_t r = J.roff; r < J.roff + J.rcnt; ++r) m0 += double(v0[P.jcells[r]]);
            for (int32_t r = J.roff; r < J.roff + J.rcnt; ++r) m1 += double(v1[P.jcells[r]]);
            m0 /= double(J.rcnt);
            m1 /= double(J.rcnt);
            if (m0 <= P.thr && m1 > P.thr) J.fire_a = n + 1 + J.delay_a;
        }
    }
}

// Advance the step counter of every live instance by k (capped at target).
static __global__ void k_advance(Tables tb, int64_t k) {
    const int32_t ni = tb.counts[2];
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ni; i += gridDim.x * blockDim.x) {
        Ctrl *c = tb.desc[i].ctrl;
        const int64_t s = c->step + k;
        c->step = s < c->target ? s : (c->step < c->target ? c->target : c->step);
    }
}

}  // namespace epdev
