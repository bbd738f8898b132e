// Host-side model of one cloth: constraint tables, the scalar PD matrix, its
// nested-dissection ordering and supernodal Cholesky factor, and the level
// schedule of the triangular solves.  Pure C++ (no HIP); built once per
// handle and uploaded by the C ABI layer.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "diffcloth.h"

namespace dc {

struct HostModel {
    // ------------------------------------------------------------ inputs
    int m = 0;                              // nodes
    std::vector<double> X;                  // [m*3] rest shape, caller order
    std::vector<double> mass;               // [m]   caller order
    double h = 0, g[3] = {0, 0, 0};
    int pd_iters = 20, fwd_max_iters = 0, adj_max_iters = 500, precision = SIM_FP64;
    double fwd_tol = 0, adj_tol = 1e-10;
    int warm_start = 0;
    double self_d = 0, self_r = 0, self_mu = 0;   // node-node contact: thickness, detection radius, friction
    int checkpoint_every = 0, adj_restart = 60, adj_solver = SIM_ADJ_ITERATIVE, adj_window = 0;
    std::vector<sim_obstacle_t> obstacles;  // mesh pointers cleared; geometry in obst_tri
    // triangle-mesh obstacles: per obstacle, per triangle its vertices a, b, c,
    // unit face normal and bounding ball (centre, radius): 16 doubles; empty
    // for planes and spheres
    std::vector<std::vector<double>> obst_tri;
    // closed meshes (every edge shared by two triangles in opposite directions):
    // a ball holding every vertex, outside of which phi > 0 without a scan
    std::vector<int> obst_closed;
    std::vector<double> obst_ball;          // per obstacle centre (3) and radius

    // ------------------------------------------------------------ constraints
    // All "norm" constraints (springs, then bending): A_c x = sum_k a_ck x_k,
    // projection onto |p| = rho_c.  Canonical order: springs in edge order,
    // then bending constraints by ascending centre node (caller ids).
    int n_edges = 0, n_bend = 0, nc = 0;
    std::vector<int32_t> edges;             // [n_edges*2]
    std::vector<int32_t> bend_center;       // [n_bend] caller ids
    std::vector<int32_t> c_ptr, c_node;     // stencil CSR, caller ids
    std::vector<double> c_coef;
    std::vector<double> rho, w, base_w, restdir;   // [nc], [nc], [nc], [nc*3]
    std::vector<int32_t> region;            // [nc] or empty
    std::vector<double> region_scale;
    std::vector<int32_t> attach;            // caller ids
    double w_att = 0, att_omega = 0, att_axis[3] = {0, 1, 0}, att_center[3] = {0, 0, 0};

    // ------------------------------------------------------------ matrices (caller order)
    // K_s = sum_c w_c a_c a_c^T + w_att sum_att e_j e_j^T ; P_s = diag(m) + h^2 K_s
    std::vector<int32_t> ks_ptr, ks_col;    // CSR, full symmetric pattern
    std::vector<double> ks_val;

    // ------------------------------------------------------------ ordering
    std::vector<int32_t> perm;              // perm[new] = old
    std::vector<int32_t> iperm;             // iperm[old] = new

    // ------------------------------------------------------------ supernodal factor (new order)
    int ns = 0;                             // supernodes
    std::vector<int32_t> sup_c0;            // [ns+1] column ranges
    std::vector<int32_t> sup_of;            // [m] supernode of each column
    std::vector<int32_t> R_ptr, R_rows;     // off-diagonal row structure of each supernode
    std::vector<int32_t> sup_level;         // [ns]
    int n_levels = 0;
    std::vector<std::vector<double>> Lblk;  // per supernode, column-major (ns_s + nR_s) x ns_s
    int64_t nnz_L = 0;

    std::string error;

    // partition of the direct adjoint's factor (same order): P's supernodes
    // with the merged top separators kept apart, cut into chunks of at most
    // lu_chunk nodes
    int lu_chunk = 42;
    std::vector<int32_t> lu_c0;             // [n_lu+1]
    std::vector<int32_t> lu_R_ptr, lu_R_rows, lu_level;
    int lu_n_levels = 0;
    int merged_nodes = 0;                   // nodes of the merged top supernode of P (0: none)

    int build(const sim_mesh_t *mesh, const sim_params_t *p);   // SIM_OK or SIM_E*
    int order_and_factor(int leaf_size, int merge_cap = 300);
    void order(int leaf_size, int merge_cap);   // ordering + symbolic structures
    int factor();                            // numeric factor on that structure
    void apply_regions();                    // w = base_w * region scale
    int assemble_ks(bool keep_pattern);      // K_s values (pattern fixed after the first call)

    // dense copy of L in the new order (tests; m small)
    void dense_L(double *out) const;
};

}  // namespace dc
