// Host-side (FP64) precompute of the tetrahedral finite-volume operator and
// the device data layout.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace ep {

enum Ordering { ORDER_RCM = 0, ORDER_MORTON = 1, ORDER_INPUT = 2 };

struct PrepIn {
    int64_t n_nodes = 0, n_tets = 0;
    const double *xyz = nullptr;       // [n_nodes*3]
    const int32_t *tets = nullptr;     // [n_tets*4]
    const double *fibre = nullptr;     // [n_tets*3]
    const double *scale = nullptr;     // [n_tets] or null
    const uint8_t *model = nullptr;    // [n_tets]
    double sigma_l = 0.17, sigma_t = 0.019, chi = 140.0, cm = 0.01;
    int ordering = ORDER_RCM;
    // bidomain: also the flux sums of the elliptic operator with the tensor
    // of conductivities (sigma_l + sigma_el, sigma_t + sigma_et)
    bool elliptic = false;
    double sigma_el = 0.0, sigma_et = 0.0;
    // a 2D medium with a time step of its own: its cells (triangles) and
    // nodes take the last internal indices, grouped by model class like
    // the tets before them
    bool split_media = false;
};

// Node gather in sliced ELL with slices of 64 nodes (one wavefront): slice
// k covers nodes [64k, 64k+64), has width w_k = (off[k+1]-off[k])/64 and
// stores entry (slot s, lane l) at off[k] + 64 s + l.  Padding entries hold
// cell 0 with weight 0.
struct PrepOut {
    int64_t n_nodes = 0, n_tets = 0;
    std::vector<int32_t> perm;        // internal cell -> caller cell
    std::vector<int32_t> iperm;       // caller cell -> internal cell
    std::vector<int64_t> sell_off;    // [n_slices+1]
    std::vector<int32_t> sell_cell;
    std::vector<double> sell_w;
    // fused cell stencil, slot-major ([slot][n_tets]; the upload converts it
    // to the device's tile-major layout), internal numbering:
    //   L_c = sum_{s<8} beta[s] vn[node[s]] + sum_{f<4} b[f] (v[nbr[f]] - v_c)
    std::vector<int32_t> cnode;       // [8][n]: own vertices, then the vertices opposite
                                      // the faces in the neighbours (triangles: 3 + 3,
                                      // slots 3 and 7 padded with coefficient 0)
    std::vector<double> cbeta;        // [8][n]
    std::vector<int32_t> cnbr;        // [4][n]: face neighbour or self on the boundary
    std::vector<double> cb;           // [4][n]
    // elliptic operator (bidomain), same nodes and neighbours, flux-sum form
    // (not divided by chi Cm V_c):  y_c = sum_s ebeta[s] x_n[node_s] +
    // sum_f eb[f] (x[nbr_f] - x_c)
    std::vector<double> ebeta;        // [8][n]
    std::vector<double> eb;           // [4][n]
    std::vector<double> vol;          // [n] tet volume or triangle area (internal order)
    std::vector<uint8_t> model;       // [n] internal order
    int64_t n_interior_faces = 0, n_boundary_faces = 0;
    int max_node_degree = 0;
    double sell_padding = 0.0;        // padded / real incidences - 1
    int64_t n_incidences = 0;         // (cell, vertex) pairs: 4 per tet, 3 per triangle
    double max_abs_L_row = 0.0;       // max_c sum of |coefficients| (stability hint)
    // with split_media: the first internal cell and node of the 2D medium
    // (n_tets / n_nodes when it has none); always: the forward-Euler bound
    // of the 2D medium's two-point operator, 1 / max_c sum_f sigma_max
    // scale_c |S_f| / (d_f chi Cm V_c) (infinite without triangles)
    int64_t cell_2d = 0, node_2d = 0;
    double dtmax_2d = 0.0;
};

// Returns an empty string on success, else the reason for EP_EINVAL.
std::string prepare(const PrepIn &in, PrepOut &out);

// ---------------------------------------------- Purkinje graph, junctions
struct PmjIn {
    int32_t node = 0;                  // Purkinje node of the junction
    int32_t cell = -1;                 // or its source cell (caller id; node ignored)
    double radius = 0.1, delay_ortho = 5.0, delay_anti = 3.0, amp = -200.0, dur = 0.5;
    int32_t two_way = 0;
};

struct PurkIn {
    int64_t n = 0, n_edges = 0;
    const double *xyz = nullptr;       // [n*3]
    const int32_t *edges = nullptr;    // [n_edges*2]
    const double *edge_scale = nullptr;  // [n_edges] conductivity multipliers >= 0, or null
    double sigma = 3.95, dt = 0.02, chi = 140.0, cm = 0.01;
    int32_t n_sub = 0;                 // <= 0: derived from the stability bound
    bool ab2 = false;                  // Adams-Bashforth 2: half the stable interval
    std::vector<PmjIn> pmjs;
};

// Vertex-centred graph operator in CSR (caller node numbering):
//   dv_i/dt += sum_{e in [off[i], off[i+1])} g[e] (v[nbr[e]] - v_i).
// Junction k stimulates the cells jcells[jroff[k] .. jroff[k+1]) (internal
// ids, listed in increasing caller id).  cpmj[c] (internal cell) is -1 or the
// start of a -1-terminated list in cpmj_list of the junctions pulsing c.
// The graph may be empty (n == 0) when every junction has a source cell.
struct PurkOut {
    int64_t n = 0;
    int32_t n_sub = 1;
    std::vector<int32_t> off, nbr;
    std::vector<double> g;
    std::vector<int32_t> jroff, jcells;
    std::vector<int32_t> jsrc;         // per junction: internal source cell, or -1 (graph node)
    // cpmj_list entries: k (pulse of junction k's region) or k | kAntiBit
    // (two-way pulse of junction k onto this cell, its source)
    std::vector<int32_t> cpmj, cpmj_list;
};
constexpr int32_t kAntiBit = 1 << 30;

std::string prepare_purkinje(const PurkIn &in, const PrepIn &tin, const PrepOut &tout,
                             PurkOut &out);

// Two-level preconditioner of the elliptic (bidomain) operator: aggregates
// of cells (internal numbering, CSR agg_off / agg_cells, agg_of per cell),
// the inverse diagonal, and the dense inverse of the aggregated operator
// (row-major n_agg x n_agg).
struct Coarse {
    int32_t n_agg = 0;
    std::vector<int32_t> agg_of, agg_off, agg_cells;
    std::vector<double> dinv, cinv;
};
std::string build_coarse(const PrepIn &in, const PrepOut &P, int target, Coarse &out);

}  // namespace ep
