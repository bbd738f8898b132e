// Device-side descriptor of one cloth handle.  Every array lives in HBM and
// uses the nested-dissection node order ("new" order); vectors of 3D
// quantities are node-major [node][xyz].  One workgroup owns one handle for
// the duration of a launch, so work buffers are private to it.
#pragma once

#include <cstddef>
#include <cstdint>

namespace dc {

constexpr int kMaxObstacles = 8;
constexpr int kBlock = 1024;         // threads per workgroup of the forward kernel (16 wavefronts)
constexpr int kBlockAdj = 1024;      // threads per workgroup of the adjoint kernel
constexpr int kSolveBatch = 4;      // 16-byte loads per lane in flight in the triangular solves of P
// Variant bits of the persistent kernels: what the host placed in LDS and, for
// the adjoint kernel, the adjoint solver (the bit value 4 means kLdsPositions
// in the forward kernel and kAdjDirect in the adjoint kernel).
constexpr int kLdsVectors = 1, kLdsUpdates = 2, kLdsPositions = 4, kAdjDirect = 4;
// variant bit of both kernels: code for triangle-mesh obstacles compiled in
// (kept out of the other variants, whose register budget it would cost)
constexpr int kMeshObst = 8;
constexpr int kTeam = 8;             // lanes cooperating on one solve row / column
constexpr int kKryM = 60;            // GMRES restart length of the adjoint fallback

// Packed solve work items (shared host/device layout).
constexpr int32_t kNoOutput = INT32_MIN;   // FwdItem.out1 of a padding row
struct FwdItem {            // forward: rows r, r + 1 (r even) of a stacked block G_s
    int32_t g;              // offset of G_s[r, 0] in gval (column stride ld, even)
    int16_t ld, kmax;       // padded column stride and number of columns used
    int32_t tbase;          // 3 * c0: first right-hand-side entry of the supernode
    int32_t out0, out1;     // per row: >= 0: 3 * (c0 + r) in the forward result; < 0: -(ubuf offset) - 1;
                            //   kNoOutput: padding row
    int32_t pad[3];
};
struct BwdItem {            // backward: columns k, k + 1 (k even) of a stacked block G_s, rows k .. ld-1
    int32_t g;              // offset of G_s[k, k] in gvalt (row-major copy, row stride st, even)
    int16_t n1, n2;         // rows k .. ns-1 (times y_s) and the nR rows of B_s (times x_{R_s})
    int32_t ybase;          // 3 * (c0 + k): y_s entry of row k and output entry of column k
    int32_t ubase;          // ubuf offset of the supernode: x_{R_s} is gathered there first
    int32_t st;             // row stride of the row-major copy
    int32_t two;            // column k + 1 exists (else padding)
    int32_t pad[2];
};
struct GatherItem {         // backward: x_{R_s} entry copied into the supernode's ubuf slot
    int32_t u;              // ubuf offset (3 doubles)
    int32_t x3;             // 3 * node; -(3 * node) - 1: a root supernode's row, read from Y
};
// the kernels read these descriptors as 16-byte / 8-byte vectors (field order as declared)
static_assert(sizeof(FwdItem) == 32 && sizeof(BwdItem) == 32 && sizeof(GatherItem) == 8, "descriptor layout");
struct RowItem {            // forward gather: t_i = b_i - sum of update entries
    int32_t i3;             // 3 * i
    int32_t p0, p1;         // range in upd_off
    int32_t pad;
};
struct SpringInc {          // node-centred spring projection: one incident spring of node i
    int32_t j;              // the other endpoint (new id)
    int32_t cs;             // spring's constraint slot c if i is its first endpoint, else ~c
    double wr;              // weight times rest length
};
static_assert(sizeof(SpringInc) == 16, "read as a 16-byte vector");

// Direct adjoint solve: one product y = M v with a column-major block M of a
// step factor, rows [a, a + nrow) (a wavefront, two rows per lane; M's column
// stride and offset are even; a short item splits its columns over groups of
// lanes).  A phase of
// the solve (one level, one kind of block) is a list of such items; its
// kAdjBatch-column batches are split evenly over the wavefronts of the workgroup.
struct AdjItem {
    int64_t moff;           // offset of M(a, 0) in a step factor
    int32_t ld;             // column stride of M
    int32_t K;              // columns of M
    int32_t vbase;          // first entry of v
    int32_t obase;          // first output entry (row a)
    int32_t nrow;           // rows of the item, <= kAdjRows
    int32_t grp;            // column groups: lanes g rp .. g rp + rp - 1 (rp = row pairs) take
                            //   columns g kAdjBatch .. of every kAdjBatch * grp (grp rp <= 64)
};
constexpr int kAdjBatch = 8;        // columns per unit of work (16-byte loads per lane in flight)
constexpr int kAdjRows = 128;       // rows per item: two per lane, read with one 16-byte load
constexpr int kAdjWaves = kBlockAdj / 64;
constexpr int kAdjHelpers = 8;      // prefetching workgroups of a single-handle direct adjoint launch
constexpr int kXcds = 8;            // workgroup i of a launch runs on XCD i mod 8
// multi-workgroup forward of one handle: at most kMwMax workgroups (all on one
// XCD), a root supernode of at most kMwRootMax columns, kMwRanges node ranges
// per workgroup; its barrier block: counter, generation, failure flag (16
// bytes), then one partial maximum and three partial counts per workgroup
constexpr int kMwMax = 16, kMwRootMax = 512, kMwRanges = 6;
constexpr int kMwMinNodes = 1200;   // nodes from which a handle runs it by default
constexpr int kMwSyncDoubles = 2 + 4 * kMwMax;
constexpr size_t kNoallocScratchBytes = size_t(16) << 20;   // device scratch of the allocation-free forward
constexpr int kMaxDevices = 64;
struct LuUpd {              // supernode s is updated by descendant d: rows [i0, i1) of R_d lie in s
    int32_t d, i0, i1;
    int32_t map;            // offset in lu_relmap of the panel rows (in s) of R_d[i0..r_d)
};
struct LuSup {              // supernode (chunk) data of the direct adjoint factor
    int32_t c0, n, r;       // first node, nodes, rows of R_s
    int32_t rptr;           // offset of R_s in sup_rows
    int32_t uoff;           // offset of u_s in the update buffer
    int32_t ldn, ldr;       // N = 3n and R = 3r rounded up to even: the row strides below
    int32_t pad;
    int64_t off;            // offset of the chunk's blocks in a step factor (doubles, even):
                            //   Dt (N x ldn) at off, Bt (N x ldr) at off + N ldn,
                            //   Ct / Vt (R x ldn) at off + N ldn + N ldr, all row-major
};

struct ObstacleDev {
    int type;                         // 0 plane, 1 sphere, 2 triangle mesh
    int n_tris;                       // mesh: triangles
    int closed;                       // mesh: closed surface (ball[] bounds it)
    double p[3], n[3], radius, mu;
    double ball[4];                   // mesh: centre and radius of a ball holding every vertex
    const double *tri;                // mesh: per triangle a, b, c, unit face normal, ball (16 doubles)
    const float *ball32;              // mesh: per triangle its ball (centre, radius) in float
};

struct SimDev {
    // ---------------------------------------------------------------- sizes, parameters
    int m;                            // nodes
    int nca;                          // active norm constraints (springs + curved bending)
    int nc_total;                     // all norm constraints (canonical numbering)
    int n_obst, na;
    int K, fwd_max_iters, adj_max_iters, mixed;
    int warm_start;                   // contact impulses start from the previous step's
    double h, fwd_tol, adj_tol;
    double g[3];
    double w_att, att_omega, att_axis[3], att_center[3];
    ObstacleDev obst[kMaxObstacles];

    // ---------------------------------------------------------------- static tables
    const double *mass;               // [m]
    const int32_t *ks_ptr, *ks_col;   // K_s CSR (new order)
    const double *ks_val;             // float64 values
    const float *ks_valf;             // float32 copy (residual SpMV in mixed precision)
    const int32_t *c_ptr, *c_node;    // active-constraint stencils (new node ids)
    const double *c_coef;
    const double *c_rho, *c_w, *c_restdir;   // [nca], [nca], [nca*3]
    const float *c_rhof, *c_wf;
    const int32_t *c_id;              // canonical index of each active constraint
    const int32_t *inc_ptr, *inc_con; // node -> active constraint incidence
    const double *inc_coef;
    const int32_t *att_node;          // [na] new ids
    const int32_t *att_of;            // [m] attachment slot or -1
    const double *att_rest;           // [na*3] rest positions (caller coordinates)

    // supernodal factor of P_s (new order): per supernode the stacked dense block
    // G_s = [L_ss^{-1}; B_s L_ss^{-1}], column-major (ns + nR) x ns
    int n_levels;
    const int32_t *lvl_rows_ptr;      // [n_levels+1] into rows (columns of each level)
    const int32_t *lvl_gat_ptr;       // [n_levels+1] into bgat
    const int32_t *lvl_bwd_ptr;       // [n_levels+1] into bwd items (column pairs of each level)
    // L2 prefetch for the forward pass (meshes whose factor of P overflows L2):
    // the solving workgroup publishes (epoch << 40 | iteration * 2 levels + phase)
    // before each level of the two triangular solves; helpers touch the blocks
    // of the next phase (forward phases read gval, backward phases gvalt)
    int64_t *fwd_pos;
    int64_t fwd_epoch;
    const int32_t *fpf_ptr;           // [2 levels + 1] into fpf: phase l < L forward level l, L + j backward level L-1-j
    const int64_t *fpf;               // [2 per range] offset and length (doubles) of a block
    int n_root_rows;                  // rows of root supernodes (no R_s): their forward product
    const int32_t *root_rows;         //   writes x_s into Y, copied to x at the end (3 i each)
    const int32_t *lvl_items_ptr;     // [n_levels+1] into fwd items
    const int32_t *lvl_team;          // [2*n_levels] lanes per item: forward, backward
    const int32_t *lvl_team_adj;      // the same for the adjoint's solves with P (one workgroup's choice)
    const RowItem *rows;
    const FwdItem *fitems;
    const BwdItem *bitems;
    const GatherItem *bgat;
    const int32_t *sup_rows;          // off-diagonal row structure R_s (concatenated)
    const double *gval;               // stacked blocks, column-major, even column stride (forward)
    const double *gvalt;              // the same blocks, row-major, even row stride (backward)
    const int32_t *upd_off;           // ubuf offsets gathered by the forward solve
    double *ubuf;                     // update vectors u_s (3 per row of R_s), HBM copy
    int n_ubuf;                       // doubles in ubuf
    // springs, node-centred (forward local step + RHS gather in one pass)
    const int32_t *sinc_ptr;          // [m+1]
    const SpringInc *sinc;
    const double *sinc_rho;           // rest length of each incidence (degenerate-length test)
    int nca_bend;                     // active (curved) bending constraints: device indices [nca - nca_bend, nca)
    const int32_t *binc_ptr, *binc_con;   // node -> active bending constraint incidence
    const double *binc_coef;

    // ---------------------------------------------------------------- state and work
    double *x, *v;                    // state x_n, v_n
    double *vk, *vk1;                 // PD iterates
    double *b0, *rhs, *ysol;          // constant rhs, rhs / gather scratch, forward-solve result
    double *f;                        // contact impulse h J^T r per node
    double *wp;                       // [nca*3] w_c p_c (forward) / projection-Jacobian products (adjoint)
    uint8_t *mode;                    // [m] contact mode of the current step
    int8_t *cobst;                    // [m] obstacle of contact nodes
    double *ubar;                     // [m*3] free velocity of the last contact update
    double *red;                      // [64] reduction scratch (per workgroup)

    // step records: slot s holds step (rec_step0 + s)
    double *rec_x;                    // [(cap+1) * m*3]: x at step rec_step0 + s
    double *rec_v;                    // [(cap+1) * m*3]
    double *rec_ubar;                 // [cap * m*3]
    uint8_t *rec_mode;                // [cap * m]
    int8_t *rec_obst;                 // [cap * m]
    int rec_cap;
    int32_t *step_info;               // [4 per step n of the rollout]: PD iterations, take-off, stick,
                                      //   slip node counts (indexed by n, not by record slot); may be null
    int rec_ring;                     // 1: every step records into slots 0 (x_n) and 1 (x_{n+1}) --
                                      //   the allocation-free forward keeps no rollout

    // adjoint buffers
    double *gx, *gv;                  // dL/dx_{n+1}, dL/dv_{n+1} -> dL/dx_n, dL/dv_n
    double *zeta, *zeta1, *zt;        // iterate, next iterate, T^T zeta
    double *adj_s, *adj_q;            // [nca], [nca*3] projection-Jacobian scale and direction at x_{n+1}
    double *adj_pq;                   // [nca*3] p - q at x_{n+1}
    double *tblk;                     // [m*9] T_j blocks (contact nodes)
    double *dw;                       // [nc_total] accumulated weight gradients (canonical)
    double *dmu;                      // [kMaxObstacles + 1]: per obstacle, then (last) self-friction
    const double *gx_steps;           // optional per-step dL/dx_n [(T+1)*m*3], new order
    double *cfr;                      // [m*8] mesh obstacles, per node the current step's contact
                                      // frame: n, phi, edge direction, region
    // external force besides gravity: step n adds fscale[n] * fext (fext nullptr:
    // none; fscale nullptr: 1 at every step), and its gradients
    const double *fext;               // [m*3] new order
    const double *fscale;             // [steps] per-step multipliers
    double *dfext;                    // [m*3] dL/dfext, new order
    double *dfscale;                  // [T] dL/dfscale[n]

    // Krylov fallback workspace (GMRES)
    double *kry;                      // [(kry_m+1) * m*3] Krylov basis
    int kry_m;                        // GMRES restart length (<= kKryM)

    // direct adjoint: per step an LU-type factor of A = M + H T^T on the
    // supernodes of P (degrees of freedom, not nodes): per supernode s with
    // N = 3 n_s, R = 3 r_s, column-major blocks D_s^{-1} (N x N), B_s = A(R_s, s)
    // after the Schur updates (R x N) and V_s = D_s^{-1} A(s, R_s) (N x R)
    int adj_direct;                   // 1: adjoint steps solved with their factors
    int ns;                           // supernodes of the factor (P's, cut into chunks)
    int lu_nlevels;                   // levels of their elimination tree
    const LuSup *lu_sup;              // [ns]
    const int32_t *lu_srows;          // R_t of every chunk (concatenated)
    const RowItem *lu_rows;           // forward gathers by level (update-buffer entries per node)
    const int32_t *lu_upd_off;        // their update-buffer offsets
    const int32_t *lu_upd_ptr;        // [ns+1] updaters of each supernode
    const LuUpd *lu_upd;
    const int32_t *lu_relmap;         // panel row in s of each row of R_d from i0 on (< n_s: in s)
    const int64_t *ks_dst;            // [nnz K_s] offset of block (i, j) in a step factor
    const int32_t *ks_ld;             // [nnz K_s] row stride there
    const int32_t *dp_ptr;            // [n_inc+1] per incidence entry (node i, constraint c):
    const int32_t *dp_ks;             //   K_s entry of (i, l) for each stencil node l of c
    const int32_t *lu_lvl;            // [2*(levels+1)]: per level start of its row gathers, x_R gathers
    const GatherItem *lu_gat;         // backward: x_{R_t} copied into the update slots of chunk t
    const AdjItem *adj_items;         // items of the phases (level l: 3l = D^{-1}, 3l+1 = B, 3l+2 = V)
    const int32_t *adj_prog;          // [3 levels * kAdjWaves * 4] per phase and wavefront: first item,
                                      //   first batch, last item, end batch (batches [.., end) of it)
    const int32_t *adj_sptr;          // [3 levels + 1] into adj_split
    const int32_t *adj_split;         // [4 per entry] item, first and last wavefront holding a part, 0
    int64_t af_size;                  // doubles per step factor
    int64_t af_ws_size;               // doubles of factorisation workspace per step
    int af_nmax;                      // largest N
    double *af;                       // step factors: slot k holds step af_step0 + k
    double *af_ws;                    // workspace per slot
    int af_step0;
    // L2 prefetch of the step factors for a single-handle adjoint launch: the
    // solving workgroup publishes its position (epoch << 40 | step * phases +
    // phase, all ones below bit 40 when done); helper workgroups on its XCD
    // touch the blocks of the next phase
    double *adj_hz;                   // direct adjoint: H T^T zeta of the last check (3m)
    double *adj_dwc;                  //   and its weight-gradient dot products (one per active constraint)
    int64_t *adj_pos;
    int64_t adj_epoch;
    const int32_t *adj_pfptr;         // [3 levels + 1] into adj_pf, by phase id
    const int64_t *adj_pf;            // [2 per range] offset and length (doubles) of a block in a step factor

    // multi-workgroup forward (one handle on mw workgroups of one XCD; 0: not
    // available): workgroup w solves whole subtrees below the root supernode
    // alone and shares the root (its columns mw_root_c0 ..)
    int mw;
    int mw_root_c0;
    const int32_t *mw_ptr;            // [4 (mw (levels - 1) + 1)]: per (workgroup, level below the
                                      //   root) ranges into mw_rows, mw_fitems, mw_bitems, mw_bgat
    const RowItem *mw_rows;
    const FwdItem *mw_fitems;
    const BwdItem *mw_bitems;
    const GatherItem *mw_bgat;
    const int32_t *mw_nodes;          // [mw][kMwRanges][2] node ranges [a, b) of each workgroup
    const int32_t *mw_win;            // [mw][4]: one subtree per workgroup, solved in LDS: its columns
                                      //   [lo, hi) and update slots [ulo, uhi) (null: vectors in HBM)
    const int32_t *mw_rootw;          // [mw][4]: the root's forward items [a, b) of each workgroup and
                                      //   where their factor entries start in gval and how many (doubles)
    int mw_root_lds;                  // 1: each workgroup copies its root entries into LDS once per launch
    int mw_root_off;                  //   (after this many doubles of dynamic LDS: the subtree window)
    uint32_t *mw_sync;                // barrier block (kMwSyncDoubles doubles)
    int64_t mw_spin;                  // wall-clock ticks (100 MHz) a barrier waits before giving up
    int mw_absent;                    // failure-handling tests only: the last workgroup returns at
                                      //   once, so every barrier wait ends at its limit

    // node-node self-collision (off when self_on == 0): pairs of mutually
    // nearest eligible nodes found on the predictor each step; the pair's
    // leader (lower caller id) runs its contact update for both nodes
    int self_on;
    double self_d, self_r2, self_mu;  // thickness, squared detection radius, friction
    const int32_t *caller_id;         // [m] caller id of each node (pair leader, ties)
    const int32_t *adj_ptr, *adj_col; // nodes sharing a constraint stencil (never paired)
    double *ybuf;                     // [m*3] predictor of the current step
    double self_inv_cell;             // 1 / grid cell size (the detection radius, widened by 1e-6)
    int self_hmask;                   // hash table size - 1 (a power of two >= 2 m)
    int32_t *self_head;               // [self_hmask + 1] first node of each hash bucket (-1: empty)
    int32_t *self_next;               // [m] next node of the same bucket
    int32_t *cand;                    // [m] nearest eligible node or -1
    int32_t *partner;                 // [m] pair partner of the current step or -1
    int32_t *rec_partner;             // [cap * m] partner per recorded step

    // run control for one launch
    int step_begin, step_end;         // forward: steps [begin, end); backward: reverse
    int rec_step0;                    // step number of record slot 0
    int64_t *counters;                // [8]: fwd iters, adj iters, fallbacks, noconv, Krylov iters
};

}  // namespace dc
