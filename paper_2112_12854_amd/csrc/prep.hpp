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
    // fused cell stencil, slot-major ([slot][n_tets]), internal numbering:
    //   L_c = sum_{s<8} beta[s] vn[node[s]] + sum_{f<4} b[f] (v[nbr[f]] - v_c)
    std::vector<int32_t> cnode;       // [8][n]: 4 own vertices, 4 opposite vertices
    std::vector<double> cbeta;        // [8][n]
    std::vector<int32_t> cnbr;        // [4][n]: face neighbour or self on the boundary
    std::vector<double> cb;           // [4][n]
    std::vector<double> vol;          // [n] tet volume (internal order)
    std::vector<uint8_t> model;       // [n] internal order
    int64_t n_interior_faces = 0, n_boundary_faces = 0;
    int max_node_degree = 0;
    double sell_padding = 0.0;        // padded / real incidences - 1
    double max_abs_L_row = 0.0;       // max_c sum of |coefficients| (stability hint)
};

// Returns an empty string on success, else the reason for EP_EINVAL.
std::string prepare(const PrepIn &in, PrepOut &out);

}  // namespace ep
