/*
 * diffcloth.h -- C ABI of the MI355X (gfx950) DiffCloth hot path.
 *
 * The library simulates cloth with Projective Dynamics (PD) and dry frictional
 * contact, and back-propagates a loss through the rollout with the adjoint
 * method of DiffCloth (Li et al., "DiffCloth: Differentiable Cloth Simulation
 * with Dry Frictional Contact", ACM TOG 2022):
 *   forward  -- per time step the PD local/global loop (Sec. 3.1, eqns
 *               pd_project, pd_global) in velocity form with contact impulses
 *               on the right-hand side (Sec. 3.2, eqns pd_velocity,
 *               pd_velocity_with_contact) and a per-node Signorini-Coulomb
 *               update (eqn contact_all);
 *   backward -- per time step the adjoint solve with the prefactored PD matrix
 *               and the per-node contact Jacobians (Sec. 4.2, eqns adjoint_v,
 *               ppr_adjoint), then the gradients with respect to the initial
 *               state, the constraint weights and the friction coefficients.
 *
 * Conventions
 *   - Every call returns an int: 0 = success, < 0 = error (SIM_E*), > 0 =
 *     success with a warning (SIM_W*).  No C++ exception crosses this ABI.
 *   - Host arrays passed to sim_create are copied; the caller keeps ownership.
 *   - "_dev" pointers are device (HBM) pointers owned by the caller; they must
 *     be valid for the sizes stated and stay valid until the call's work on
 *     the handle's stream has finished.  Positions, velocities and gradients
 *     are node-major float64 arrays [n_nodes][3] in the caller's node order.
 *   - All device memory the handle needs comes from the caller's allocator
 *     callback (e.g. the PyTorch caching allocator) or, when it is NULL, from
 *     hipMalloc; it is returned in sim_destroy.
 *   - All device work is enqueued on the stream given to sim_create (NULL =
 *     the default stream).  Calls that return data to the host synchronise
 *     that stream.
 *   - A handle is not thread-safe; use one handle per thread or lock.
 */
#ifndef DIFFCLOTH_H
#define DIFFCLOTH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
#define SIM_OK               0
#define SIM_EINVAL          -1   /* bad mesh or parameters                              */
#define SIM_ENOTSPD         -2   /* a Cholesky pivot of the PD matrix is not positive   */
#define SIM_ENOMEM          -3   /* allocation failed                                   */
#define SIM_ENONFINITE      -4   /* NaN / Inf in inputs or state                        */
#define SIM_ESTATE          -5   /* call out of order (backward before forward, ...)    */
#define SIM_EHIP            -6   /* a HIP runtime call failed                           */
#define SIM_ESCRATCH        -7   /* the mesh needs more device scratch than
                                    sim_forward_noalloc has (16 MiB)                   */
#define SIM_ESYNC           -8   /* a multi-workgroup forward launch gave up waiting at
                                    a barrier (its workgroups were not all resident
                                    in time); the rollout is not recorded              */
#define SIM_WADJ_FALLBACK    1   /* >= 1 adjoint step needed the fallback solver        */
#define SIM_WADJ_NOCONV      2   /* >= 1 adjoint step did not reach its tolerance       */
#define SIM_WADJ_NONFINITE   3   /* the state gradients overflowed (not finite)         */

#define SIM_PLANE            0
#define SIM_SPHERE           1
#define SIM_MESH             2

#define SIM_FP64             0   /* every step in float64                               */
#define SIM_MIXED            1   /* float32 local projections, projection Jacobians and
                                    residual SpMV; float64 solves, contact, accumulation */

#define SIM_ADJ_ITERATIVE    0   /* adjoint steps by the paper's fixed point (Sec. 4.2)
                                    with the prefactored P; GMRES when it stalls      */
#define SIM_ADJ_DIRECT       1   /* adjoint steps by a direct factorisation of each
                                    step's matrix (all steps factored in parallel)    */

#define SIM_MODE_FREE        0   /* node not in the contact set                          */
#define SIM_MODE_TAKEOFF     1
#define SIM_MODE_STICK       2
#define SIM_MODE_SLIP        3

/* ---------------------------------------------------------------- types */
typedef struct sim sim_t;

/* Static obstacle.  Plane: {x : n.(x - p) = 0}, signed distance n.(x - p)
 * with unit normal n.  Sphere: centre p, radius r, signed distance |x - p| - r.
 * Mesh (the triangulated obstacles of Sec. 5.1's discretized-sphere study):
 * n_tris triangles over n_verts vertices (host arrays verts [n_verts*3],
 * tris [n_tris*3], copied by sim_create; at most 65536 triangles, none
 * degenerate); the outward side of triangle t is that of
 * (v1 - v0) x (v2 - v0).  A point's closest triangle (ties to the lowest index)
 * gives its frame: on the triangle's face the face normal and the plane
 * distance; at an edge or vertex with closest point c, the direction of
 * x - c and |x - c|, signed by the side of the triangle's face.  The scan over
 * all triangles suits obstacles of a few thousand triangles.  mu is the
 * Coulomb friction coefficient of any type; the mesh fields are ignored for
 * planes and spheres. */
typedef struct {
    int32_t type;          /* SIM_PLANE, SIM_SPHERE or SIM_MESH */
    double  p[3];
    double  n[3];
    double  radius;
    double  mu;
    int32_t n_verts;       /* SIM_MESH */
    int32_t n_tris;
    const double  *verts;
    const int32_t *tris;
} sim_obstacle_t;

/* Triangle mesh.  X is the rest shape, also the default initial state.
 * Springs are the unique triangle edges (a < b, sorted lexicographically)
 * unless an explicit edge list is given.  Attachment targets are the rest
 * positions rotated by attach_omega * t about attach_axis through
 * attach_center (omega = 0: fixed pins). */
typedef struct {
    int32_t        n_nodes;
    const double  *X;              /* [n_nodes*3] */
    int32_t        n_tris;
    const int32_t *tris;           /* [n_tris*3]  */
    int32_t        n_edges;        /* 0: extract from tris */
    const int32_t *edges;          /* [n_edges*2] or NULL  */
    int32_t        n_attach;
    const int32_t *attach;         /* [n_attach] node ids  */
    double         attach_omega;
    double         attach_axis[3];
    double         attach_center[3];
} sim_mesh_t;

/* Physical and solver parameters.
 *  h, pd_iters     time step (s) and PD local/global iterations per step;
 *  fwd_tol         > 0: iterate each step until max|v^{k+1} - v^k| <= fwd_tol
 *                  (m/s) or fwd_max_iters; <= 0: exactly pd_iters iterations;
 *  node_mass       [n_nodes] lumped masses (kg), all > 0;
 *  edge_stiffness  [n_edges] spring weights (N/m) in the spring order above;
 *  bend_weight     quadratic-bending weight (cotangent Laplacian, one
 *                  constraint per interior vertex);
 *  attach_weight   attachment constraint weight (N/m);
 *  edge_region / bend_region / region_scale: optional; spring e uses
 *                  edge_stiffness[e] * region_scale[edge_region[e]], the
 *                  bending constraint at node j bend_weight *
 *                  region_scale[bend_region[j]] (NULL: scale 1);
 *  adj_tol         adjoint stop rule max|zeta^{k+1}-zeta^k| <= adj_tol*max|zeta^{k+1}|;
 *  adj_max_iters   fixed-point iterations before the GMRES fallback, and the
 *                  GMRES iteration budget;
 *  adj_restart     GMRES restart length, 1..60 (0: 60);
 *  adj_solver      SIM_ADJ_ITERATIVE or SIM_ADJ_DIRECT.  Direct: every step's
 *                  adjoint matrix M + H T^T is factored (supernodes of P,
 *                  pivoting inside each diagonal block), all steps of a
 *                  rollout (or checkpoint segment) at once, one workgroup per
 *                  step; each step is then solved with its factor and refined
 *                  against the matrix until the normwise backward error
 *                  |gbar - A zeta| / (|A| |zeta| + |gbar|) (max norms) is at
 *                  most adj_tol (at most adj_max_iters solves).  Device memory: one factor
 *                  per step of the segment (sim_stats_t.adj_factor_bytes each);
 *  adj_window      direct adjoint: factor at most this many steps at a time
 *                  (the window nearest the end first, then its solves, then
 *                  the next window); 0: all steps of the segment at once;
 *  checkpoint_every  0: keep every step's record for the backward pass;
 *                  k > 0: keep the state every k steps and recompute segments;
 *  warm_start      1: each step's contact iteration starts from the previous
 *                  step's impulses on the nodes of its contact set (0: from
 *                  zero impulses); the converged state does not depend on it,
 *                  a fixed pd_iters result does.  Checkpoints keep the
 *                  impulses, so replayed segments reproduce their records.
 *  self_thickness  node-node self-collision (Sec. 4.2, Extensions; 0: off):
 *                  thickness d (m).  Each step, on the inertial predictor y,
 *                  every node outside the obstacle contact set takes as
 *                  partner its nearest node j with |y_i - y_j| <= self_radius
 *                  (0: d) that shares no spring or bending stencil with it and
 *                  sits elsewhere at x_n (ties to the lower caller id);
 *                  mutually nearest nodes form a pair.  The pair's normal is
 *                  n = (x_i - x_j)/|x_i - x_j| at x_n (i the lower caller id),
 *                  its gap |x_i - x_j| - d; the law of eqn contact_all acts on
 *                  v_i - v_j with the reduced mass m_i m_j / (m_i + m_j) and
 *                  friction self_mu, impulse +f on i and -f on j.  Needs
 *                  SIM_ADJ_ITERATIVE (SIM_EINVAL otherwise: a pair's adjoint
 *                  block lies outside the direct factor's pattern).  The pair
 *                  search hashes the predictors into a uniform grid of cells
 *                  no smaller than the detection radius (27 cells per node).
 *  (The tolerance rule of fwd_tol measures the change of the velocities and
 *  of the contact impulses in velocity units, |f^{k+1} - f^k| / m_j.) */
typedef struct {
    double                h;
    int32_t               pd_iters;
    double                fwd_tol;
    int32_t               fwd_max_iters;
    double                gravity[3];
    const double         *node_mass;
    const double         *edge_stiffness;
    double                bend_weight;
    double                attach_weight;
    const int32_t        *edge_region;
    const int32_t        *bend_region;
    const double         *region_scale;
    int32_t               n_regions;
    int32_t               n_obstacles;      /* <= 8 */
    const sim_obstacle_t *obstacles;
    int32_t               precision;        /* SIM_FP64 or SIM_MIXED */
    double                adj_tol;
    int32_t               adj_max_iters;
    int32_t               checkpoint_every;
    int32_t               adj_restart;
    int32_t               adj_solver;
    int32_t               adj_window;
    int32_t               warm_start;
    double                self_thickness;
    double                self_radius;
    double                self_mu;
} sim_params_t;

/* Gradient outputs (caller-allocated device arrays; any may be NULL). */
typedef struct {
    double *dx0;      /* [n_nodes*3] dL/dx_0                                   */
    double *dv0;      /* [n_nodes*3] dL/dv_0                                   */
    double *dw_edge;  /* [n_edges]   dL/d(spring weight)                       */
    double *dw_bend;  /* [n_nodes]   dL/d(bending weight of the constraint at
                                     node j); 0 for boundary nodes            */
    double *dregion;  /* [n_regions] dL/d(region_scale)                        */
    double *dmu;      /* [n_obstacles] dL/d(mu)                                */
    double *dforce;   /* [n_nodes*3] dL/dF of the external force field F (see
                         sim_set_external_force); zeros when no force is set  */
    double *dforce_scale; /* [T] dL/ds_n of its per-step multipliers over the
                         T recorded steps; zeros when no force is set          */
    double *dmu_self; /* [1] dL/d(self_mu) of node-node contacts (0 when off)  */
} sim_grads_t;

typedef struct {
    int32_t n_nodes, n_edges, n_bend, n_constraints_active;
    int64_t nnz_P, nnz_L;           /* scalar PD matrix and its Cholesky factor  */
    int32_t n_supernodes, n_levels; /* supernodal elimination tree              */
    int32_t steps_recorded;
    int64_t fwd_iters_total;        /* PD iterations of the last forward        */
    int64_t adj_iters_total;        /* fixed-point iterations of the last backward */
    int32_t adj_fallbacks;          /* steps solved by the fallback             */
    int32_t adj_noconv;             /* steps that missed the tolerance          */
    int64_t device_bytes;           /* device memory held by the handle         */
    int64_t adj_krylov_total;       /* GMRES iterations of the fallback         */
    int64_t factor_bytes;           /* bytes of the stacked factor blocks       */
    int64_t lds_forward, lds_backward; /* dynamic LDS per workgroup (0: vectors in HBM) */
    int64_t adj_factor_bytes;       /* direct adjoint: bytes of one step's factor */
    int64_t adj_pivot_perturbed;    /* direct adjoint: pivots raised to the floor in the last backward */
    int32_t fwd_launches;           /* forward kernel launches of the last sim_forward (chunks
                                       overlapped with the direct adjoint's step factorisations,
                                       or checkpoint segments) */
    int32_t lds_flags_fwd;          /* kernel variant of a single-handle forward launch: data kept in
                                       LDS (1 PD iterates / solve vectors, 2 the solve's update
                                       buffer, 4 the positions x_n; 0: everything in HBM) */
    int32_t lds_flags_bwd;          /* the same for the adjoint kernel (1 and 2 only)             */
    int32_t fwd_iters_max;          /* most PD iterations taken by one step of the recorded rollout */
    int64_t mode_counts[4];         /* node-steps of the recorded rollout in each contact mode,
                                       indexed by SIM_MODE_* (free, take-off, stick, slip)       */
    double  fwd_ms, bwd_ms;         /* device time of the last sim_forward / sim_backward on the
                                       handle's stream (HIP events; 0 before the first call)    */
    int32_t fwd_workgroups;         /* workgroups of a single-handle forward launch (> 1: the
                                       multi-workgroup kernel, subtrees of the elimination tree per
                                       workgroup)                                               */
    int32_t pad;
} sim_stats_t;

typedef void *(*sim_alloc_fn)(size_t bytes, void *ctx);
typedef void  (*sim_free_fn)(void *ptr, void *ctx);

/* ---------------------------------------------------------------- calls */

/* Builds the constraint set (springs, bending, attachments; eqn pd_project),
 * assembles the scalar PD matrix P_s with P = P_s (x) I_3 (eqn pd_global),
 * orders it by nested dissection, factors it (supernodal Cholesky, float64,
 * "prefactorized at the beginning of the simulation", Sec. 3.1) and uploads
 * everything.  Returns SIM_EINVAL on bad inputs, SIM_ENOTSPD on a
 * non-positive pivot, SIM_ENOMEM / SIM_EHIP on device failures. */
int sim_create(const sim_mesh_t *mesh, const sim_params_t *params, void *hip_stream,
               sim_alloc_fn alloc, sim_free_fn free_fn, void *alloc_ctx, sim_t **out);

/* sim_create in two parts, for callers that prepare handles off their
 * serving thread:
 *  sim_plan_create      the host part -- constraint tables, the PD matrix, the
 *                       ordering and the Cholesky factor (Sec. 3.1) -- with no
 *                       GPU call; distinct plans may be built on different
 *                       threads at the same time.  Errors as sim_create's host
 *                       checks (SIM_EINVAL, SIM_ENONFINITE, SIM_ENOTSPD, SIM_ENOMEM).
 *  sim_create_from_plan the device part (tables uploaded, kernels configured)
 *                       on the given stream and allocator, as sim_create; it
 *                       takes the plan over on success (do not destroy it then)
 *                       and leaves it usable on failure.  Device set-ups are
 *                       serialised within a process.
 *  sim_plan_destroy     releases a plan that was not used (NULL is ignored).
 * sim_create is sim_plan_create followed by sim_create_from_plan. */
typedef struct sim_plan sim_plan_t;
int  sim_plan_create(const sim_mesh_t *mesh, const sim_params_t *params, sim_plan_t **out);
int  sim_create_from_plan(sim_plan_t *plan, void *hip_stream, sim_alloc_fn alloc, sim_free_fn free_fn,
                          void *alloc_ctx, sim_t **out);
void sim_plan_destroy(sim_plan_t *plan);

/* External force besides gravity, part of f_ext in the implicit Euler step
 * (Sec. 3.1): during step n node j receives scale[n] * force[j] newtons, which
 * enters the inertial predictor, the initial guess and the constant part of the
 * right-hand side b_hat (eqn pd_velocity); the applications' wind models
 * (Sec. 6: a sinusoidal gust times a direction, per-node coefficients) and the
 * time-invariant per-node control forces of Sec. 5.2 are of this form.
 *  force_dev   device [n_nodes*3] (caller order), copied on the handle's
 *              stream; NULL removes the external force;
 *  scale_host  host [n_scale] per-step multipliers s_n, copied before return;
 *              NULL: s_n = 1 at every step (n_scale ignored); n_scale >= 1
 *              otherwise.
 * A later forward pass over more than n_scale steps returns SIM_EINVAL.
 * The backward pass then also returns dL/dF = h sum_n s_n z_n and
 * dL/ds_n = h F . z_n (z_n = T^T zeta of step n; sim_grads_t.dforce,
 * dforce_scale).  Invalidates any recorded rollout.  SIM_EINVAL on a NULL
 * handle, n_scale < 1 with a scale, or a non-finite multiplier (the device
 * field is not inspected: non-finite forces surface as non-finite states and
 * the backward pass's SIM_WADJ_NONFINITE); SIM_ENOMEM / SIM_EHIP on device
 * failures. */
int sim_set_external_force(sim_t *sim, const double *force_dev, int32_t n_scale, const double *scale_host);

/* Sets the initial state (device arrays [n_nodes*3], caller order).  NULL x0
 * = rest shape; NULL v0 = zero.  Invalidates any recorded rollout. */
int sim_set_state(sim_t *sim, const double *x0_dev, const double *v0_dev);

/* Changes the material of a handle and refactors P (Sec. 3.1: P depends on
 * the constraint weights only, so a weight change is a numeric refactor on
 * the handle's ordering and symbolic structure; the mesh, masses and
 * obstacles' geometry stay).  Host arrays, each NULL = keep:
 *   edge_stiffness [n_edges], bend_weight (one scalar), region_scale
 *   [n_regions] (SIM_EINVAL if the handle has no regions), obstacle_mu
 *   [n_obstacles] (friction only; no refactor).
 * Weights must be finite and >= 0 (SIM_ENONFINITE / SIM_EINVAL); a weight
 * that was exactly 0 at sim_create and becomes nonzero changes the sparsity
 * pattern of P and is rejected with SIM_EINVAL; a non-positive pivot returns
 * SIM_ENOTSPD.  On any error the handle keeps its previous material.
 * Invalidates any recorded rollout; synchronises the handle's stream. */
int sim_set_material(sim_t *sim, const double *edge_stiffness, const double *bend_weight,
                     const double *region_scale, const double *obstacle_mu);

/* Runs n_steps implicit-Euler steps with dry frictional contact from the
 * initial state and records what the backward pass needs.  Optional outputs:
 * x_traj_dev [(n_steps+1)*n_nodes*3] (x_0 .. x_T), xT_dev, vT_dev [n_nodes*3]. */
int sim_forward(sim_t *sim, int32_t n_steps, double *x_traj_dev, double *xT_dev, double *vT_dev);

/* Back-propagates dL/dx_T (and optionally dL/dv_T and per-step dL/dx_n,
 * [(T+1)*n_nodes*3], entry n is added when the pass reaches x_n) through the
 * recorded rollout.  Returns SIM_ESTATE if no rollout is recorded; warnings
 * (the gradients are written): SIM_WADJ_NONFINITE if the state gradients
 * overflowed (the adjoint of a step amplifies when its matrix is far from
 * positive definite, e.g. after a truncated forward iteration), else
 * SIM_WADJ_NOCONV / SIM_WADJ_FALLBACK if an adjoint step missed its
 * tolerance / fell back. */
int sim_backward(sim_t *sim, const double *dL_dxT_dev, const double *dL_dvT_dev,
                 const double *dL_dx_steps_dev, const sim_grads_t *out);

/* One adjoint step at recorded step n (0 <= n < T): given dL/dx_{n+1} and
 * dL/dv_{n+1}, writes dL/dx_n, dL/dv_n and this step's weight / friction
 * gradients (dw_edge, dw_bend, dmu of `out`; the others are ignored). */
int sim_adjoint_step(sim_t *sim, int32_t n, const double *gx_dev, const double *gv_dev,
                     double *dx_dev, double *dv_dev, const sim_grads_t *out);

/* Recorded state (x_n, v_n) of the last forward pass, 0 <= n <= T, written
 * to caller device arrays [n_nodes*3] (either may be NULL). */
int sim_state(const sim_t *sim, int32_t n, double *x_dev, double *v_dev);

/* Contact modes (SIM_MODE_*) of recorded step n, caller node order, host array [n_nodes]. */
int sim_modes(const sim_t *sim, int32_t n, uint8_t *modes_host);

/* Node-node contact pairs of recorded step n (Sec. 4.2, Extensions): host
 * array partner_host [n_nodes], caller node order and ids; -1 for a node in no
 * pair.  A pair's nodes carry its contact mode in sim_modes.  With
 * self-collision off every entry is -1.  SIM_ESTATE without a recorded
 * rollout, SIM_EINVAL for n out of range. */
int sim_self_pairs(const sim_t *sim, int32_t n, int32_t *partner_host);

/* Counters of the last forward pass and backward pass, sizes of the handle's
 * tables and factors (synchronises the handle's stream). */
int sim_stats(const sim_t *sim, sim_stats_t *out);

/* Per-step record of the last forward pass, 0 <= n < T (host array out[4]):
 * PD iterations of step n and the number of its nodes in take-off, stick and
 * slip mode (the contact set of step n is their sum; Sec. 3.2).  SIM_ESTATE
 * without a recorded rollout, SIM_EINVAL for n out of range. */
int sim_step_stats(const sim_t *sim, int32_t n, int32_t *out);

/* Batched forward / backward of independent handles in one persistent launch
 * (one workgroup per handle; handles may differ in size and step count).  All
 * handles must share the first handle's stream and precision, and for the
 * backward call its adj_solver (else SIM_EINVAL).  Per-handle arguments are
 * arrays of length n (entries may be NULL where the single call allows it). */
int sim_batch_forward(sim_t *const *sims, int32_t n, const int32_t *n_steps,
                      double *const *xT_dev, double *const *vT_dev);
int sim_batch_backward(sim_t *const *sims, int32_t n, const double *const *dL_dxT_dev,
                       const sim_grads_t *out);

/* Releases the device memory a handle holds only for a rollout: step records,
 * checkpoints, the per-step loss buffer, the direct adjoint's step factors and
 * work lists (the next rollout allocates them again).  The mesh tables and the
 * factor of P stay.  Drops the recorded rollout (as sim_set_state); waits for
 * the handle's stream. */
int sim_trim(sim_t *sim);

/* Continuous batching.  A job on a handle is a forward rollout followed by its
 * backward pass, run in chunks of steps so that handles can join and leave a
 * running batch between launches (the results are bitwise those of
 * sim_forward / sim_backward on the same handle).  Handles used this way keep
 * every step's record (checkpoint_every must be 0).
 *   sim_job_forward   arms a forward pass of n_steps from the initial state;
 *   sim_job_backward  arms the backward pass of the finished forward pass
 *                     (dL/dx_T, optional dL/dv_T; device arrays, caller order);
 *   sim_batch_advance advances every listed handle's armed phase by up to
 *                     steps[i] steps: one launch for all forward chunks on the
 *                     first handle's stream and, for the backward chunks, the
 *                     step factorisations (direct adjoint) and one launch on
 *                     backward_stream (NULL: the same stream); all handles must
 *                     share the first handle's stream, precision and
 *                     adj_solver (else SIM_EINVAL).  It
 *                     returns when both streams are done; left[i] (host, may be
 *                     NULL) receives the steps still to run in the phase (0:
 *                     phase finished; x_T then via sim_state, gradients via
 *                     sim_job_grads).  Handles without an armed phase are an
 *                     error (SIM_ESTATE);
 *   sim_job_grads     writes the gradients of a finished backward pass, with
 *                     the return convention of sim_backward. */
int sim_job_forward(sim_t *sim, int32_t n_steps);
int sim_job_backward(sim_t *sim, const double *dL_dxT_dev, const double *dL_dvT_dev);
int sim_batch_advance(sim_t *const *sims, int32_t n, const int32_t *steps, void *backward_stream, int32_t *left);
int sim_job_grads(sim_t *sim, const sim_grads_t *out);

/* Allocation-free variant of sim_forward, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  It runs n_steps from the handle's initial state
 * (sim_set_state) exactly as sim_forward does -- the same kernels, bitwise the
 * same x_T and v_T -- and writes x_T, v_T (device [n_nodes*3], caller order,
 * both required).  It records nothing for a backward pass and leaves the
 * handle's recorded rollout, if any, as it was.  Its per-step work memory (PD
 * iterates, right-hand side, the solve's update buffer, impulses, contact
 * modes and frames, the running state) lives in one 16 MiB device array per
 * GPU that the library holds until the process ends; no call of this function
 * allocates, frees, synchronises or issues a memset (it only enqueues copies
 * and kernels on the handle's stream and returns).  Every call on one GPU uses
 * that GPU's array: calls that overlap on one GPU (other streams, other
 * threads) race and their results are undefined.  Returns SIM_ESCRATCH when
 * the mesh needs more than the array holds (sim_noalloc_scratch_bytes tells
 * the need; about 400 bytes per node plus the solve's update buffer),
 * SIM_EINVAL on bad arguments or when external-force multipliers run out,
 * SIM_EHIP on a HIP error. */
int sim_forward_noalloc(sim_t *sim, int32_t n_steps, double *xT_dev, double *vT_dev);

/* Device scratch bytes sim_forward_noalloc needs for this handle (-1: NULL). */
int64_t sim_noalloc_scratch_bytes(const sim_t *sim);

/* Host-only analysis (no GPU needed): builds the constraint set, the PD
 * matrix, the ordering and the Cholesky factor exactly as sim_create does and
 * reports their sizes.  perm_out [n_nodes] (may be NULL) receives the
 * elimination order (new -> caller node id); dense_L_out [n_nodes^2]
 * (row-major, may be NULL) the factor L with P_s[perm][:, perm] = L L^T when
 * n_nodes <= max_dense. */
int sim_analyze(const sim_mesh_t *mesh, const sim_params_t *params, int32_t leaf_size, sim_stats_t *stats,
                int32_t *perm_out, double *dense_L_out, int32_t max_dense);

void        sim_destroy(sim_t *sim);
const char *sim_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* DIFFCLOTH_H */
