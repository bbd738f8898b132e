// C ABI of the DiffCloth hot path: handle lifetime, device tables, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <vector>

#include "diffcloth.h"
#include "host_model.h"
#include "sim_dev.h"

namespace dc {
hipError_t launch_forward(const SimDev *d_sims, int n, bool mixed, size_t lds, int flags, int helpers, bool mesh,
                          hipStream_t st);
hipError_t launch_backward(const SimDev *d_sims, int n, bool mixed, size_t lds, int flags, int helpers, bool mesh,
                           hipStream_t st);
hipError_t configure_lds(size_t fwd_bytes, size_t bwd_bytes);
hipError_t kernel_static_lds(size_t *fwd, size_t *bwd);
hipError_t launch_permute3(const double *in, double *out, const int32_t *perm, int m, bool to_caller, hipStream_t st);
hipError_t launch_modes(const uint8_t *in, uint8_t *out, const int32_t *perm, int m, hipStream_t st);
hipError_t launch_region_grad(const double *dw, const double *base_w, const int32_t *region, int nc, int nreg,
                              double *out, hipStream_t st);
hipError_t launch_scatter_bend(const double *dw, const int32_t *centers, int n_edges, int n_bend, double *out,
                               hipStream_t st);
hipError_t launch_fill(double *p, double v, int64_t n, hipStream_t st);
hipError_t launch_adj_assemble(const SimDev *d_sims, const int32_t *work, int nblocks, hipStream_t st);
hipError_t launch_adj_factor_level(const SimDev *d_sims, const int32_t *work, int nblocks, int nmax, hipStream_t st);
hipError_t noalloc_scratch(void **out);
hipError_t launch_forward_mw(const SimDev *d, int W, bool mixed, bool mesh, bool lw, size_t lds, int threads,
                             hipStream_t st);
hipError_t configure_mw_lds(size_t bytes);
}  // namespace dc

using namespace dc;

struct sim {
    HostModel hm;
    hipStream_t stream = nullptr;
    sim_alloc_fn alloc = nullptr;
    sim_free_fn free_fn = nullptr;
    void *ctx = nullptr;
    std::vector<std::pair<void *, int64_t>> owned;   // every device allocation of the handle and its size
    int64_t bytes = 0;                  // their total (what sim_stats reports)
    SimDev *batch_desc = nullptr;       // descriptors of the batched launches this handle leads
    bool mw_used = false;               // a multi-workgroup forward ran since the last mw_check
    size_t mw_lds = 0;                  // dynamic LDS of its workgroups
    bool mw_lw = false;                 // each of them solves its subtree in LDS (else vectors in HBM)
    SimDev hd_noalloc{};                // descriptor of the allocation-free forward (copied to the
                                        //   device scratch on every call; lives as long as the handle)
    int step_info_cap = 0;              // steps the per-step record (hd.step_info) can hold
    hipEvent_t tev[4] = {nullptr, nullptr, nullptr, nullptr};   // forward start / end, backward start / end
    bool tev_fwd = false, tev_bwd = false;                       // recorded by the last calls
    size_t batch_desc_cap = 0;          //   (capacity in descriptors; reused across calls)

    SimDev hd{};                        // host copy of the descriptor
    SimDev *dd = nullptr;               // device copy (one element)
    int32_t *d_perm = nullptr;          // new -> caller
    double *rest_x = nullptr;           // rest shape, new order
    double *start_x = nullptr, *start_v = nullptr;  // state a forward pass starts from
    double *ckpt = nullptr;             // checkpoints: [n_seg][3][m*3] (x, v, contact impulses)
    int ckpt_cap = 0;
    double *gsteps = nullptr;           // per-step loss gradients, new order
    double *fext_buf = nullptr;         // external force field, new order
    double *fscale_buf = nullptr;       // its per-step multipliers
    int n_fscale = 0, fscale_cap = 0;
    double *dfext_buf = nullptr;        // dL/d(force field), new order
    double *dfscale_buf = nullptr;      // dL/d(multiplier) per step
    int dfscale_cap = 0;
    int gsteps_cap = 0;
    const double *d_basew = nullptr;
    const int32_t *d_region = nullptr;
    const int32_t *d_bend_centers = nullptr;
    uint8_t *d_modes_tmp = nullptr;
    int T = -1;                         // steps of the recorded rollout (-1: none)
    int phase = 0;                      // continuous batching: 0 idle, 1 forward armed, 2 forward done,
                                        // 3 backward armed, 4 backward done
    int cursor = 0, target = 0;         // next step (forward) / steps still to go back (backward)
    int64_t counters_host[8] = {0};
    int nca = 0;
    int af_cap = 0;                     // step factors allocated (direct adjoint)
    int n_ubuf_bwd = 0;                 // update-buffer doubles the backward kernel needs
    std::vector<std::vector<int32_t>> lvl_sn;   // supernodes of each elimination level (adjoint factor)
    std::vector<int32_t> lvl_nmax;      // largest diagonal block (DoF) of each of those levels
    std::vector<int32_t> h_work;        // factorisation work lists (host copy)
    int32_t *d_work = nullptr;          // and their device copy
    size_t work_cap = 0;
    // step factorisations overlapped with the forward pass (direct adjoint,
    // no checkpoints, no adjoint window): a second stream factors each chunk
    // of steps once the forward pass has recorded it
    hipStream_t fac_stream = nullptr;
    hipEvent_t fac_ev = nullptr, fac_done = nullptr;
    SimDev hd_fac{};                    // descriptor the overlapped factorisation reads,
    SimDev *dd_fac = nullptr;           //   and its device copy
    int prefactored = 0;                // steps [0, prefactored) of the recorded rollout are factored
    int fwd_launches = 0;               // forward launches of the last sim_forward
    std::vector<int32_t> corder;        // device constraint slot -> canonical constraint id
    int64_t factor_bytes = 0;
    size_t lds_fwd = 0, lds_bwd = 0;   // dynamic LDS of the two kernels
    int flags_fwd = 0, flags_bwd = 0;  // what lives in LDS (kLds* bits)
    size_t static_fwd = 0, static_bwd = 0, max_lds = 0;
    int cus = 0;                        // compute units of the device
};

namespace {

int hip_err(hipError_t e) { return e == hipSuccess ? SIM_OK : SIM_EHIP; }

// Nested-dissection leaf size (nodes per leaf supernode) of a mesh of m
// nodes: 128 where the multi-workgroup forward runs by default (its solves
// pay per level: at 40 x 40, leaves of 32 / 64 / 128 nodes give 5 / 4 / 3
// levels and 641 / 684 / 744 cloth steps/s), else 32.  DIFFCLOTH_LEAF
// overrides it for experiments.
int leaf_size_default(int m) {
    const char *e = std::getenv("DIFFCLOTH_LEAF");
    const int v = e ? std::atoi(e) : 0;
    return v >= 4 && v <= 256 ? v : (m >= kMwMinNodes ? 128 : 32);
}

// Largest merged top supernode of P (nodes); DIFFCLOTH_MERGE overrides it for
// experiments (0: no merging).
int merge_cap_default() {
    const char *e = std::getenv("DIFFCLOTH_MERGE");
    const int v = e ? std::atoi(e) : -1;
    return v >= 0 && v <= 4096 ? v : 300;
}

// Prefetch workgroups per handle of a forward launch: 2 when the largest
// handle's factor of P (both copies) passes 3 MB (a quarter of an XCD's L2
// is left for the rest), if every workgroup of the launch can be resident.
int fwd_helpers(sim *const *sims, int n) {
    const char *e = std::getenv("DIFFCLOTH_FWD_HELPERS");
    int h = e ? std::atoi(e) : -1;
    if (h < 0) {
        int64_t mx = 0;
        for (int i = 0; i < n; ++i) mx = std::max(mx, 2 * sims[i]->factor_bytes);
        h = mx > (3 << 20) ? 2 : 0;
    }
    h = std::min(h, 7);
    return h > 0 && (int64_t)n * (1 + h) <= sims[0]->cus ? h : 0;
}

// Workgroups of a single handle's forward launch (the multi-workgroup kernel
// when the elimination tree allows it): DIFFCLOTH_FWD_WGS, 0 or 1 = one;
// unset: as many as the root has subtrees (at most 16) from kMwMinNodes on --
// below that its barriers cost more than the split saves (24 x 24 nodes: 39
// against 27 us per PD iteration; 40 x 40: 61 against 73; 64 x 64: 136
// against 340, measured on MI355X).
int mw_workgroups_default(int m) {
    const char *e = std::getenv("DIFFCLOTH_FWD_WGS");
    const int v = e ? std::atoi(e) : -1;
    if (v >= 0) return std::min(v, kMwMax);
    return m >= kMwMinNodes ? kMwMax : 0;
}

// Whether a multi-workgroup forward solves each workgroup's subtree in LDS
// (DIFFCLOTH_MW_LDS=0: vectors in HBM).
bool mw_lds_default() {
    const char *e = std::getenv("DIFFCLOTH_MW_LDS");
    return !(e && *e == '0');
}

// Whether each workgroup of a multi-workgroup forward keeps its run of the
// root's stored inverse in LDS (DIFFCLOTH_MW_ROOT_LDS=0: read from L2).
bool mw_root_lds_default() {
    const char *e = std::getenv("DIFFCLOTH_MW_ROOT_LDS");
    return !(e && *e == '0');
}

// wall-clock ticks (100 MHz) a multi-workgroup barrier waits before giving up
int64_t mw_spin_default() {
    const char *e = std::getenv("DIFFCLOTH_MW_SPIN");
    const long long v = e ? std::atoll(e) : -1;
    return v >= 0 ? (int64_t)v : (int64_t)100000000;       // 1 s
}

// Threads per workgroup of the multi-workgroup forward (a multiple of 64 up
// to 1024; DIFFCLOTH_MW_THREADS).  The work of a subtree is split into items
// and nodes that any thread count covers in the same arithmetic, so the count
// changes timing only.
int mw_threads_default() {
    const char *e = std::getenv("DIFFCLOTH_MW_THREADS");
    const int v = e ? std::atoi(e) : 0;
    return v >= 64 && v <= 1024 && v % 64 == 0 ? v : 1024;
}

// prefetch workgroups of a single-handle direct adjoint launch (0: none)
int adj_helpers_default() {
    const char *e = std::getenv("DIFFCLOTH_ADJ_HELPERS");
    const int v = e ? std::atoi(e) : -1;
    return v >= 0 && v <= 16 ? v : kAdjHelpers;
}

void *dev_alloc(sim *s, size_t bytes) {
    if (bytes == 0) bytes = 8;
    bytes = (bytes + 255) & ~size_t(255);
    void *p = nullptr;
    if (s->alloc) {
        p = s->alloc(bytes, s->ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (!p) throw std::bad_alloc();
    s->owned.emplace_back(p, (int64_t)bytes);
    s->bytes += (int64_t)bytes;
    return p;
}

void dev_release(sim *s, void *p) {
    if (!p) return;
    auto it = std::find_if(s->owned.begin(), s->owned.end(), [p](const auto &e) { return e.first == p; });
    if (it != s->owned.end()) {
        s->bytes -= it->second;
        s->owned.erase(it);
    }
    if (s->free_fn) s->free_fn(p, s->ctx);
    else (void)hipFree(p);
}

// Device room for n descriptors of a batched launch led by handle s, kept
// between calls (grown when a batch is larger than any before it).
SimDev *batch_descs(sim *s, size_t n) {
    if (n > s->batch_desc_cap) {
        const size_t cap = std::max<size_t>(n, 2 * s->batch_desc_cap);
        dev_release(s, s->batch_desc);
        s->batch_desc = nullptr;
        s->batch_desc_cap = 0;
        s->batch_desc = (SimDev *)dev_alloc(s, cap * sizeof(SimDev));
        s->batch_desc_cap = cap;
    }
    return s->batch_desc;
}

template <class T>
T *upload(sim *s, const std::vector<T> &v) {
    T *d = (T *)dev_alloc(s, v.size() * sizeof(T));
    if (!v.empty() && hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s->stream) != hipSuccess)
        throw std::runtime_error("hip copy");
    return d;
}

template <class T>
T *zeros(sim *s, size_t n) {
    T *d = (T *)dev_alloc(s, n * sizeof(T));
    if (hipMemsetAsync(d, 0, std::max<size_t>(n, 1) * sizeof(T), s->stream) != hipSuccess)
        throw std::runtime_error("hip memset");
    return d;
}

// Column groups of a direct-solve item of nrow rows and K columns: as many
// lane groups (a power of two, at most 8) as fit a wavefront beside its row
// pairs and have columns to take.
int adj_groups(int nrow, int K) {
    const int rp = (nrow + 1) / 2;
    int g = 1;
    while (g < 8 && 2 * g * rp <= 64 && g * kAdjBatch < K) g *= 2;
    return g;
}

// Splits the column batches of one phase of the direct adjoint solve into
// kAdjWaves contiguous runs of (nearly) equal length, in item order; a cut
// inside an item moves to the item's boundary when that is at most one batch
// away.  Appends the items, each wavefront's run (first item, first batch,
// last item, end batch) and the items whose batches span several
// wavefronts (their parts are summed in wavefront order; wavefronts with an
// empty run in between hold no part).
void balance_phase(const std::vector<AdjItem> &ph, std::vector<AdjItem> &items, std::vector<int32_t> &prog,
                   std::vector<int32_t> &split, std::vector<int32_t> &sptr) {
    const int base = (int)items.size(), ni = (int)ph.size();
    std::vector<int64_t> pre(ni + 1, 0);                  // first batch of each item
    for (int i = 0; i < ni; ++i) {
        const int span = kAdjBatch * ph[i].grp;
        pre[i + 1] = pre[i] + std::max(1, (ph[i].K + span - 1) / span);
    }
    const int64_t total = pre[ni];
    std::vector<int64_t> cut(kAdjWaves + 1, 0);
    cut[kAdjWaves] = total;
    for (int w = 1; w < kAdjWaves; ++w) {
        int64_t c = (total * w + kAdjWaves / 2) / kAdjWaves;
        const int i = (int)(std::upper_bound(pre.begin(), pre.end(), c) - pre.begin()) - 1;   // item holding batch c
        if (i < ni) {
            if (c - pre[i] <= 1) c = pre[i];
            else if (pre[i + 1] - c <= 1) c = pre[i + 1];
        }
        cut[w] = std::max(c, cut[w - 1]);
    }
    auto locate = [&](int64_t c, int &item, int &batch) {           // batch c as (item, batch in item)
        if (c >= total) { item = ni; batch = 0; return; }
        item = (int)(std::upper_bound(pre.begin(), pre.end(), c) - pre.begin()) - 1;
        batch = (int)(c - pre[item]);
    };
    std::vector<int> first_item(kAdjWaves);
    for (int w = 0; w < kAdjWaves; ++w) {
        int i0, b0, i1, b1;
        locate(cut[w], i0, b0);
        locate(cut[w + 1], i1, b1);
        first_item[w] = i0;
        for (int v : {base + i0, b0, base + i1, b1}) prog.push_back(v);
    }
    for (int i = 0; i < ni; ++i) {
        int wa = -1, wb = -1;
        for (int w = 0; w < kAdjWaves; ++w)
            if (cut[w + 1] > cut[w] && cut[w] < pre[i + 1] && cut[w + 1] > pre[i]) { if (wa < 0) wa = w; wb = w; }
        if (wa >= 0 && wb > wa)
            for (int v : {base + i, wa, wb, 0}) split.push_back(v);
    }
    sptr.push_back((int32_t)(split.size() / 4));
    items.insert(items.end(), ph.begin(), ph.end());
}

// variant bits of an adjoint launch: LDS placement plus the handle's solver
int bwd_variant(const sim *s, int lds_flags) { return (lds_flags & 3) | (s->hd.adj_direct ? kAdjDirect : 0); }

// A handle of the launch has a triangle-mesh obstacle: the kernels' mesh variant.
bool has_mesh(sim *const *hs, int n) {
    for (int i = 0; i < n; ++i)
        for (const sim_obstacle_t &o : hs[i]->hm.obstacles)
            if (o.type == SIM_MESH) return true;
    return false;
}

size_t lds_bytes(const sim *s, int flags, bool fwd) {
    const size_t m3 = 3 * (size_t)s->hd.m;
    size_t b = 0;
    if (flags & kLdsVectors) b += 2 * m3;
    if (flags & kLdsUpdates) b += (size_t)(fwd ? s->hd.n_ubuf : s->n_ubuf_bwd);
    if (fwd && (flags & kLdsPositions)) b += m3;
    return b * sizeof(double);
}

// Kinds of data the LDS placement may use: DIFFCLOTH_LDS (a mask of kLdsVectors
// = 1, kLdsUpdates = 2, kLdsPositions = 4) restricts the greedy choice below,
// so that tests can run every kernel variant on a small mesh; unset: all.
int lds_allowed() {
    const char *e = std::getenv("DIFFCLOTH_LDS");
    if (!e || !*e) return 7;
    const int v = std::atoi(e);
    return v >= 0 && v <= 7 ? v : 7;
}

// Greedy placement: add each allowed kind of data to LDS while it still fits.
void plan_lds(sim *s, int &flags, size_t &bytes, bool fwd) {
    const size_t avail = s->max_lds > (fwd ? s->static_fwd : s->static_bwd)
                             ? s->max_lds - (fwd ? s->static_fwd : s->static_bwd) : 0;
    const int allowed = lds_allowed();
    flags = 0;
    for (int bit : {kLdsVectors, kLdsUpdates, kLdsPositions}) {
        if ((!fwd && bit == kLdsPositions) || !(allowed & bit)) continue;
        if (lds_bytes(s, flags | bit, fwd) <= avail) flags |= bit;
    }
    bytes = lds_bytes(s, flags, fwd);
}

// K_s in the new order: pattern (kp, kc) and values in both precisions.
void ks_new_order(const HostModel &hm, std::vector<int32_t> &kp, std::vector<int32_t> &kc, std::vector<double> &kv,
                  std::vector<float> &kvf) {
    const int m = hm.m;
    kp.assign(1, 0);
    kc.clear();
    kv.clear();
    kvf.clear();
    for (int i = 0; i < m; ++i) {
        const int o = hm.perm[i];
        std::vector<std::pair<int, double>> row;
        for (int k = hm.ks_ptr[o]; k < hm.ks_ptr[o + 1]; ++k) row.push_back({hm.iperm[hm.ks_col[k]], hm.ks_val[k]});
        std::sort(row.begin(), row.end());
        for (auto &pr : row) { kc.push_back(pr.first); kv.push_back(pr.second); kvf.push_back((float)pr.second); }
        kp.push_back((int32_t)kc.size());
    }
}

// Supernodal factor stacked per supernode as G_s = [L_ss^{-1}; B_s L_ss^{-1}]
// (ld = ns + nR rows, ns columns) with B_s = L(R_s, s) the off-diagonal block:
//   forward  y_s = L_ss^{-1} t_s and u_s = B_s y_s = (B_s L_ss^{-1}) t_s in one product,
//   backward x_s = L_ss^{-T} y_s - (B_s L_ss^{-1})^T x_{R_s}.
// A root supernode (nR = 0) stores instead the inverse of its diagonal block,
// (L_ss L_ss^T)^{-1} = L_ss^{-T} L_ss^{-1} (dense, symmetric): its forward
// product gives x_s at once and it has no backward product.
// Stored item by item, in the order the solve's work items read them, so that
// the lanes of an item read consecutive 16-byte words:
//   gval (offset goff[s]): per forward row pair (r, r + 1), for k = 0 ..
//     fwd_pair_cols - 1 the pair {G[r][k], G[r+1][k]} (a row past the block: 0);
//   gvalt (offset gofft[s], none for a root): per backward column pair
//     (k, k + 1), for rows j = k .. ld - 1 the pair {G[j][k], G[j][k+1]}
//     (a column past the block: 0).
// Every item starts at an even offset.
int fwd_pair_cols(int nsz, int r, bool root) { return root ? nsz : r + 1 < nsz ? r + 2 : nsz; }

void stacked_factor(const HostModel &hm, std::vector<double> &gval, std::vector<double> &gvalt,
                    std::vector<int64_t> &goff, std::vector<int64_t> &gofft) {
    const int ns = hm.ns;
    goff.assign(ns, 0);
    gofft.assign(ns, 0);
    gval.clear();
    gvalt.clear();
    std::vector<double> Gd;
    for (int sn = 0; sn < ns; ++sn) {
        const int nsz = hm.sup_c0[sn + 1] - hm.sup_c0[sn];
        const int nR = hm.R_ptr[sn + 1] - hm.R_ptr[sn], nrow = nsz + nR;
        const std::vector<double> &F = hm.Lblk[sn];       // column-major nrow x nsz, L_ss on top
        std::vector<double> inv((size_t)nsz * nsz, 0.0);   // row-major L_ss^{-1}
        for (int j = 0; j < nsz; ++j) {
            for (int i = j; i < nsz; ++i) {
                double acc = i == j ? 1.0 : 0.0;
                for (int k = j; k < i; ++k) acc -= F[(size_t)k * nrow + i] * inv[(size_t)k * nsz + j];
                inv[(size_t)i * nsz + j] = acc / F[(size_t)i * nrow + i];
            }
        }
        const int ldp = nrow + (nrow & 1);
        Gd.assign((size_t)ldp * nsz, 0.0);                  // the block, column-major, zero padding row
        double *G = Gd.data();
        if (nR == 0) {                                      // root: (L L^T)^{-1}
            for (int k = 0; k < nsz; ++k)
                for (int r = 0; r < nsz; ++r) {
                    double acc = 0.0;
                    for (int j = std::max(r, k); j < nsz; ++j) acc += inv[(size_t)j * nsz + r] * inv[(size_t)j * nsz + k];
                    G[(size_t)k * ldp + r] = acc;
                }
        } else {
            for (int k = 0; k < nsz; ++k) {
                for (int r = k; r < nsz; ++r) G[(size_t)k * ldp + r] = inv[(size_t)r * nsz + k];
                for (int q = 0; q < nR; ++q) {
                    double acc = 0.0;
                    for (int j = k; j < nsz; ++j) acc += F[(size_t)j * nrow + nsz + q] * inv[(size_t)j * nsz + k];
                    G[(size_t)k * ldp + nsz + q] = acc;
                }
            }
        }
        goff[sn] = (int64_t)gval.size();
        for (int r = 0; r < nrow; r += 2) {
            const int km = fwd_pair_cols(nsz, r, nR == 0);
            for (int k = 0; k < km; ++k) {
                gval.push_back(G[(size_t)k * ldp + r]);
                gval.push_back(G[(size_t)k * ldp + r + 1]);     // r + 1 = ldp - 1: the zero padding row
            }
        }
        gofft[sn] = (int64_t)gvalt.size();
        if (nR == 0) continue;
        for (int k = 0; k < nsz; k += 2)
            for (int j = k; j < nrow; ++j) {
                gvalt.push_back(G[(size_t)k * ldp + j]);
                gvalt.push_back(k + 1 < nsz ? G[(size_t)(k + 1) * ldp + j] : 0.0);
            }
    }
}

// Weights of the device constraint slots (canonical ids in corder).
void slot_weights(const HostModel &hm, const std::vector<int32_t> &corder, std::vector<double> &cw,
                  std::vector<float> &cwf) {
    cw.clear();
    cwf.clear();
    for (int c : corder) {
        cw.push_back(hm.w[c]);
        cwf.push_back((float)hm.w[c]);
    }
}

// Node-centred springs (active springs only): every node lists the springs
// it ends, with the spring's other data inlined.
void spring_incidence(const HostModel &hm, const std::vector<int32_t> &corder, int nca, std::vector<int32_t> &sp,
                      std::vector<SpringInc> &sv, std::vector<double> &srho, int &nca_bend) {
    const int m = hm.m;
    std::vector<std::vector<std::pair<SpringInc, double>>> sl(m);
    nca_bend = 0;
    for (int c = 0; c < nca; ++c) {
        const int canon = corder[c];
        if (canon < hm.n_edges) {
            const int a = hm.iperm[hm.c_node[hm.c_ptr[canon]]], b = hm.iperm[hm.c_node[hm.c_ptr[canon] + 1]];
            const double w0 = hm.w[canon], r0 = hm.rho[canon];
            sl[a].push_back({SpringInc{b, c, w0 * r0}, r0});
            sl[b].push_back({SpringInc{a, ~c, w0 * r0}, r0});
        } else {
            ++nca_bend;
        }
    }
    sp.assign(1, 0);
    sv.clear();
    srho.clear();
    for (int i = 0; i < m; ++i) {
        for (const auto &e : sl[i]) {
            sv.push_back(e.first);
            srho.push_back(e.second);
        }
        sp.push_back((int32_t)sv.size());
    }
}

// Build every device table from the host model and upload it.
void build_device(sim *s) {
    HostModel &hm = s->hm;
    const int m = hm.m;
    SimDev &D = s->hd;
    D = SimDev{};
    D.m = m;
    D.nc_total = hm.nc;
    D.n_obst = (int)hm.obstacles.size();
    D.na = (int)hm.attach.size();
    D.K = hm.pd_iters;
    D.fwd_max_iters = hm.fwd_max_iters;
    D.adj_max_iters = hm.adj_max_iters;
    D.mixed = hm.precision == SIM_MIXED;
    D.h = hm.h;
    D.fwd_tol = hm.fwd_tol;
    D.mw_spin = mw_spin_default();
    {
        const char *e = std::getenv("DIFFCLOTH_MW_TEST_ABSENT");   // failure-handling tests
        D.mw_absent = e && std::atoi(e) > 0 ? 1 : 0;
    }
    D.warm_start = hm.warm_start;
    D.self_on = hm.self_d > 0 ? 1 : 0;
    D.self_d = hm.self_d;
    D.self_r2 = hm.self_r * hm.self_r;
    D.self_mu = hm.self_mu;
    D.adj_tol = hm.adj_tol;
    for (int d = 0; d < 3; ++d) {
        D.g[d] = hm.g[d];
        D.att_axis[d] = hm.att_axis[d];
        D.att_center[d] = hm.att_center[d];
    }
    D.w_att = hm.w_att;
    D.att_omega = hm.att_omega;
    for (int o = 0; o < D.n_obst; ++o) {
        const sim_obstacle_t &ob = hm.obstacles[o];
        D.obst[o].type = ob.type;
        for (int d = 0; d < 3; ++d) { D.obst[o].p[d] = ob.p[d]; D.obst[o].n[d] = ob.n[d]; }
        D.obst[o].radius = ob.radius;
        D.obst[o].mu = ob.mu;
        D.obst[o].n_tris = ob.type == SIM_MESH ? ob.n_tris : 0;
        D.obst[o].closed = ob.type == SIM_MESH ? hm.obst_closed[o] : 0;
        for (int d = 0; d < 4; ++d) D.obst[o].ball[d] = hm.obst_ball.empty() ? 0.0 : hm.obst_ball[4 * o + d];
        D.obst[o].tri = ob.type == SIM_MESH ? upload(s, hm.obst_tri[o]) : nullptr;
        if (ob.type == SIM_MESH) {       // float copy of the triangles' balls for the culling sweeps
            const std::vector<double> &tr = hm.obst_tri[o];
            std::vector<float> b32(4 * (size_t)ob.n_tris);
            for (int t = 0; t < ob.n_tris; ++t) {
                for (int d = 0; d < 4; ++d) b32[4 * t + d] = (float)tr[16 * t + 12 + d];
                b32[4 * t + 3] = std::nextafter((float)tr[16 * t + 15], INFINITY);   // radius rounded up
            }
            D.obst[o].ball32 = upload(s, b32);
        }
        if (ob.type == SIM_MESH && !D.cfr) D.cfr = zeros<double>(s, 8 * (size_t)m);
    }
    const auto &perm = hm.perm, &iperm = hm.iperm;
    // masses
    std::vector<double> mass(m);
    for (int i = 0; i < m; ++i) mass[i] = hm.mass[perm[i]];
    D.mass = upload(s, mass);
    // K_s in the new order
    std::vector<int32_t> kp, kc;
    std::vector<double> kv;
    std::vector<float> kvf;
    ks_new_order(hm, kp, kc, kv, kvf);
    D.ks_ptr = upload(s, kp);
    D.ks_col = upload(s, kc);
    D.ks_val = upload(s, kv);
    D.ks_valf = upload(s, kvf);
    // constraints: active (rho > 0) first, then the rest; canonical ids kept
    std::vector<int32_t> order;
    for (int c = 0; c < hm.nc; ++c)
        if (hm.rho[c] > 0) order.push_back(c);
    const int nca = (int)order.size();
    for (int c = 0; c < hm.nc; ++c)
        if (!(hm.rho[c] > 0)) order.push_back(c);
    D.nca = nca;
    s->nca = nca;
    s->corder = order;
    std::vector<int32_t> cp(1, 0), cn, cid;
    std::vector<double> cc, crho, cw, crd;
    std::vector<float> crhof, cwf;
    slot_weights(hm, order, cw, cwf);
    for (int c : order) {
        for (int k = hm.c_ptr[c]; k < hm.c_ptr[c + 1]; ++k) {
            cn.push_back(iperm[hm.c_node[k]]);
            cc.push_back(hm.c_coef[k]);
        }
        cp.push_back((int32_t)cn.size());
        cid.push_back(c);
        crho.push_back(hm.rho[c]);
        crhof.push_back((float)hm.rho[c]);
        for (int d = 0; d < 3; ++d) crd.push_back(hm.restdir[3 * c + d]);
    }
    D.c_ptr = upload(s, cp);
    D.c_node = upload(s, cn);
    D.c_coef = upload(s, cc);
    D.c_rho = upload(s, crho);
    D.c_w = upload(s, cw);
    D.c_rhof = upload(s, crhof);
    D.c_wf = upload(s, cwf);
    D.c_restdir = upload(s, crd);
    D.c_id = upload(s, cid);
    // node -> active constraint incidence
    std::vector<std::vector<std::pair<int, double>>> inc(m);
    for (int c = 0; c < nca; ++c)
        for (int k = cp[c]; k < cp[c + 1]; ++k) inc[cn[k]].push_back({c, cc[k]});
    std::vector<int32_t> ip(1, 0), ic;
    std::vector<double> icf;
    for (int i = 0; i < m; ++i) {
        for (auto &pr : inc[i]) { ic.push_back(pr.first); icf.push_back(pr.second); }
        ip.push_back((int32_t)ic.size());
    }
    D.inc_ptr = upload(s, ip);
    D.inc_con = upload(s, ic);
    D.inc_coef = upload(s, icf);
    // attachments
    std::vector<int32_t> an, aof(m, -1);
    std::vector<double> arest;
    for (size_t a = 0; a < hm.attach.size(); ++a) {
        const int o = hm.attach[a];
        an.push_back(iperm[o]);
        aof[iperm[o]] = (int32_t)a;
        for (int d = 0; d < 3; ++d) arest.push_back(hm.X[3 * o + d]);
    }
    D.att_node = upload(s, an);
    D.att_of = upload(s, aof);
    D.att_rest = upload(s, arest);
    // supernodal factor (stacked blocks) and the solve's update-vector layout
    const int ns = hm.ns;
    std::vector<double> gval, gvalt;
    std::vector<int64_t> goff, gofft;
    stacked_factor(hm, gval, gvalt, goff, gofft);
    std::vector<int32_t> sc0(ns), sns(ns), snr(ns), rptr(ns + 1, 0), rows, uoff(ns + 1, 0);
    for (int sn = 0; sn < ns; ++sn) {
        sc0[sn] = hm.sup_c0[sn];
        sns[sn] = hm.sup_c0[sn + 1] - hm.sup_c0[sn];
        snr[sn] = hm.R_ptr[sn + 1] - hm.R_ptr[sn];
        for (int q = 0; q < snr[sn]; ++q) rows.push_back(hm.R_rows[hm.R_ptr[sn] + q]);
        rptr[sn + 1] = (int32_t)rows.size();
        uoff[sn + 1] = uoff[sn] + 3 * snr[sn];
    }
    // per column: the update-vector entries it gathers in the forward solve (ascending supernode)
    std::vector<std::vector<int32_t>> upd(m);
    for (int sn = 0; sn < ns; ++sn)
        for (int q = 0; q < snr[sn]; ++q) upd[rows[rptr[sn] + q]].push_back(uoff[sn] + 3 * q);
    std::vector<int32_t> up(1, 0), uo;
    for (int i = 0; i < m; ++i) {
        uo.insert(uo.end(), upd[i].begin(), upd[i].end());
        up.push_back((int32_t)uo.size());
    }
    if (gval.size() >= (size_t)INT32_MAX || gvalt.size() >= (size_t)INT32_MAX || uoff[ns] >= INT32_MAX / 2)
        throw std::runtime_error("factor too large");
    // level work lists (packed) and lanes per item
    std::vector<int32_t> lrp(hm.n_levels + 1, 0), lip(hm.n_levels + 1, 0), lgp(hm.n_levels + 1, 0),
        lbp(hm.n_levels + 1, 0), team(2 * hm.n_levels, 1), team_adj(2 * hm.n_levels, 1);
    std::vector<RowItem> ritems;
    std::vector<BwdItem> bitems;
    std::vector<GatherItem> bgat;
    std::vector<int32_t> root_rows;                 // 3 i for the rows of root supernodes
    std::vector<char> is_root_row(m, 0);
    for (int sn = 0; sn < ns; ++sn)
        if (snr[sn] == 0)
            for (int c = sc0[sn]; c < sc0[sn] + sns[sn]; ++c) is_root_row[c] = 1;
    std::vector<FwdItem> fitems;
    std::vector<int> lfmax(hm.n_levels, 1), lbmax(hm.n_levels, 1);   // longest item per level
    auto pick_team = [](int items, int maxlen) {
        int best = 1;
        double best_cost = 1e300;
        for (int tl = 1; tl <= 64; tl *= 2) {
            const int passes = (items * tl + kBlock - 1) / kBlock;
            // dependent round trips: kSolveBatch loads per lane in flight per batch
            const double cost = passes * ((maxlen + kSolveBatch * tl - 1) / (kSolveBatch * tl) +
                                          0.5 * __builtin_ctz(tl) + 1.0);
            if (cost < best_cost) { best_cost = cost; best = tl; }
        }
        return best;
    };
    // work items of one supernode (gather rows, forward row pairs, backward
    // column pairs, backward gathers); returns its longest forward / backward item
    auto emit = [&](int sn, std::vector<RowItem> &ri, std::vector<FwdItem> &fi, std::vector<BwdItem> &bi,
                    std::vector<GatherItem> &gi, int &fmx, int &bmx) {
        const int c0 = sc0[sn], nsz = sns[sn], ld = nsz + snr[sn];
        if (ld >= 32768) throw std::runtime_error("supernode too large");
        const int ldp = ld + (ld & 1), nszp = nsz + (nsz & 1);
        const bool root = snr[sn] == 0;
        (void)ldp;
        (void)nszp;
        for (int k = 0; k < nsz; ++k) ri.push_back(RowItem{3 * (c0 + k), up[c0 + k], up[c0 + k + 1], 0});
        int64_t bo = gofft[sn];                       // items' pairs stored one after another (stacked_factor)
        for (int k = 0; k < nsz && !root; k += 2) {  // columns k, k + 1
            BwdItem b{};
            b.g = (int32_t)bo;
            b.n1 = (int16_t)(nsz - k);
            b.n2 = (int16_t)snr[sn];
            b.ybase = 3 * (c0 + k);
            b.ubase = uoff[sn];
            b.st = 2;                                 // consecutive rows: consecutive 16-byte pairs
            b.two = k + 1 < nsz;
            bi.push_back(b);
            bo += 2 * (int64_t)(ld - k);
            bmx = std::max(bmx, ld - k);
        }
        for (int q = 0; q < snr[sn]; ++q) {        // x of a root's rows is still in Y (encoded -(3i) - 1)
            const int i = rows[rptr[sn] + q];
            gi.push_back(GatherItem{uoff[sn] + 3 * q, is_root_row[i] ? -3 * i - 1 : 3 * i});
        }
        auto out_of = [&](int r) { return r < nsz ? 3 * (c0 + r) : -(uoff[sn] + 3 * (r - nsz)) - 1; };
        int64_t fo = goff[sn];
        for (int r = 0; r < ld; r += 2) {           // rows r, r + 1
            FwdItem f{};
            f.g = (int32_t)fo;
            f.ld = 2;                                 // consecutive columns: consecutive 16-byte pairs
            f.kmax = (int16_t)fwd_pair_cols(nsz, r, root);
            fo += 2 * (int64_t)f.kmax;
            f.tbase = 3 * c0;
            f.out0 = out_of(r);
            f.out1 = r + 1 < ld ? out_of(r + 1) : kNoOutput;
            fi.push_back(f);
            fmx = std::max(fmx, (int)f.kmax);
        }
    };
    for (int l = 0; l < hm.n_levels; ++l) {
        int fmax = 1, bmax = 1;
        for (int sn = 0; sn < ns; ++sn) {
            if (hm.sup_level[sn] != l) continue;
            if (snr[sn] == 0)
                for (int k = 0; k < sns[sn]; ++k) root_rows.push_back(3 * (sc0[sn] + k));
            emit(sn, ritems, fitems, bitems, bgat, fmax, bmax);
        }
        lrp[l + 1] = (int32_t)ritems.size();
        lip[l + 1] = (int32_t)fitems.size();
        lgp[l + 1] = (int32_t)bgat.size();
        lbp[l + 1] = (int32_t)bitems.size();
        lfmax[l] = fmax;
        lbmax[l] = bmax;
        team_adj[2 * l] = team[2 * l] = pick_team(lip[l + 1] - lip[l], fmax);
        team_adj[2 * l + 1] = team[2 * l + 1] = pick_team(lbp[l + 1] - lbp[l], bmax);
        // a large root (the stored inverse) of a mesh the multi-workgroup
        // forward serves: 16 lanes per row pair, so that each workgroup's run of
        // a few row pairs is short (the one-workgroup kernel, which must sum in
        // the same order, pays about 15 % more on this product)
        if (l == hm.n_levels - 1 && m >= kMwMinNodes && fmax >= 128) team[2 * l] = std::max(team[2 * l], 16);
    }
    // Multi-workgroup forward: with one root supernode (the merged top
    // separators) whose children head subtrees of their own columns, W
    // workgroups each solve whole subtrees alone and share the root.  Subtrees
    // go to the least loaded workgroup (factor entries, largest first); every
    // workgroup also owns a slice of the root's columns.
    D.mw = 0;
    {
        const int L = hm.n_levels;
        std::vector<int> parent(ns, -1);
        for (int sn = 0; sn < ns; ++sn)
            if (snr[sn] > 0) parent[sn] = hm.sup_of[rows[rptr[sn]]];
        int nroot = 0, root = -1;
        for (int sn = 0; sn < ns; ++sn)
            if (parent[sn] < 0) { ++nroot; root = sn; }
        std::vector<int> kids;
        for (int sn = 0; sn < ns; ++sn)
            if (parent[sn] >= 0 && parent[sn] == root) kids.push_back(sn);
        // a mesh the multi-workgroup forward serves by default: lanes per item
        // of the levels below the root sized for one workgroup's share of a
        // level's items (whether or not that kernel runs: the one-workgroup
        // kernel takes the same teams, so both sum in the same order)
        if (m >= kMwMinNodes && nroot == 1 && kids.size() >= 2) {
            const int Wt = std::min<int>((int)kids.size(), kMwMax);
            for (int l = 0; l + 1 < L; ++l) {
                team[2 * l] = pick_team((lip[l + 1] - lip[l] + Wt - 1) / Wt, lfmax[l]);
                team[2 * l + 1] = pick_team((lbp[l + 1] - lbp[l] + Wt - 1) / Wt, lbmax[l]);
            }
        }
        const int want = mw_workgroups_default(m);
        int W = std::min<int>({want, (int)kids.size(), kMwMax});
        bool ok = nroot == 1 && L >= 2 && W >= 2 && sns[root] <= kMwRootMax && hm.sup_level[root] == L - 1;
        for (int sn = 0; sn < ns && ok; ++sn)
            if (sn != root && hm.sup_level[sn] == L - 1) ok = false;   // the root alone on the top level
        if (ok) {
            std::vector<int> head(ns, -1);          // root child heading each supernode's subtree
            std::vector<int> kid_of(ns, -1);
            for (size_t k = 0; k < kids.size(); ++k) kid_of[kids[k]] = (int)k;
            for (int sn = 0; sn < ns; ++sn) {
                int t = sn;
                while (t >= 0 && parent[t] >= 0 && parent[t] != root) t = parent[t];
                head[sn] = (t >= 0 && parent[t] == root) ? kid_of[t] : -1;
            }
            std::vector<double> wt(kids.size(), 0.0);
            std::vector<int> lo(kids.size(), INT32_MAX), hi(kids.size(), -1), cnt(kids.size(), 0);
            for (int sn = 0; sn < ns; ++sn) {
                const int k = head[sn];
                if (k < 0) continue;
                wt[k] += (double)sns[sn] * (sns[sn] + snr[sn]);
                lo[k] = std::min(lo[k], sc0[sn]);
                hi[k] = std::max(hi[k], sc0[sn] + sns[sn]);
                cnt[k] += sns[sn];
            }
            for (size_t k = 0; k < kids.size(); ++k)
                if (hi[k] - lo[k] != cnt[k]) ok = false;     // a subtree's columns are contiguous
            std::vector<int> order(kids.size()), owner(kids.size(), 0);
            for (size_t k = 0; k < kids.size(); ++k) order[k] = (int)k;
            std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return wt[a] > wt[b]; });
            std::vector<double> load(W, 0.0);
            std::vector<int> nsub(W, 0);
            for (int k : order) {
                const int wbest = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                owner[k] = wbest;
                load[wbest] += wt[k];
                ++nsub[wbest];
            }
            for (int w = 0; w < W; ++w)
                if (nsub[w] + 1 > kMwRanges) ok = false;
            if (ok) {
                std::vector<int32_t> nodes((size_t)W * kMwRanges * 2, 0);
                std::vector<int> used(W, 0);
                for (size_t k = 0; k < kids.size(); ++k) {
                    const int w = owner[k], r = used[w]++;
                    nodes[2 * ((size_t)w * kMwRanges + r)] = lo[k];
                    nodes[2 * ((size_t)w * kMwRanges + r) + 1] = hi[k];
                }
                const int rc0 = sc0[root], rn = sns[root];
                for (int w = 0; w < W; ++w) {           // the root's columns, in W slices
                    const int r = used[w]++;
                    nodes[2 * ((size_t)w * kMwRanges + r)] = rc0 + (int)((int64_t)rn * w / W);
                    nodes[2 * ((size_t)w * kMwRanges + r) + 1] = rc0 + (int)((int64_t)rn * (w + 1) / W);
                }
                std::vector<RowItem> mri;
                std::vector<FwdItem> mfi;
                std::vector<BwdItem> mbi;
                std::vector<GatherItem> mgi;
                const int Q = W * (L - 1);
                std::vector<int32_t> ptr(4 * ((size_t)Q + 1), 0);     // rows, fwd, bwd, gather
                for (int w = 0; w < W; ++w)
                    for (int l = 0; l < L - 1; ++l) {
                        int fmx = 1, bmx = 1;
                        for (int sn = 0; sn < ns; ++sn)
                            if (hm.sup_level[sn] == l && head[sn] >= 0 && owner[head[sn]] == w)
                                emit(sn, mri, mfi, mbi, mgi, fmx, bmx);
                        const int q = w * (L - 1) + l + 1;
                        ptr[q] = (int32_t)mri.size();
                        ptr[(Q + 1) + q] = (int32_t)mfi.size();
                        ptr[2 * (Q + 1) + q] = (int32_t)mbi.size();
                        ptr[3 * (Q + 1) + q] = (int32_t)mgi.size();
                    }
                // one subtree per workgroup: its columns and update slots, solved in LDS
                bool one = (int)kids.size() == W;
                std::vector<int32_t> win(4 * (size_t)W, 0);
                size_t need = 0;
                for (size_t k = 0; k < kids.size() && one; ++k) {
                    int ulo = INT32_MAX, uhi = -1, nu = 0;
                    for (int sn = 0; sn < ns; ++sn)
                        if (head[sn] == (int)k) {
                            ulo = std::min(ulo, uoff[sn]);
                            uhi = std::max(uhi, uoff[sn + 1]);
                            nu += uoff[sn + 1] - uoff[sn];
                        }
                    if (uhi - ulo != nu) { one = false; break; }
                    const int w = owner[k];
                    win[4 * w] = lo[k];
                    win[4 * w + 1] = hi[k];
                    win[4 * w + 2] = ulo;
                    win[4 * w + 3] = uhi;
                    need = std::max(need, (size_t)(6 * (hi[k] - lo[k]) + (uhi - ulo)) * sizeof(double));
                }
                // the root's forward items (row pairs of its stored inverse) in W
                // contiguous runs, and where each run's factor entries lie in gval
                std::vector<int32_t> rootw(4 * (size_t)W, 0);
                size_t rootc = 0;
                {
                    const int i0 = lip[L - 1], nit = lip[L] - lip[L - 1];
                    for (int w = 0; w < W; ++w) {
                        const int a = i0 + (int)((int64_t)nit * w / W), b = i0 + (int)((int64_t)nit * (w + 1) / W);
                        rootw[4 * w] = a;
                        rootw[4 * w + 1] = b;
                        if (b > a) {        // an item's pairs follow the previous item's (emit)
                            const int64_t g0 = fitems[a].g;
                            const int64_t g1 = (int64_t)fitems[b - 1].g + 2 * (int64_t)fitems[b - 1].kmax;
                            rootw[4 * w + 2] = (int32_t)g0;
                            rootw[4 * w + 3] = (int32_t)(g1 - g0);
                            rootc = std::max(rootc, (size_t)(g1 - g0) * sizeof(double));
                        }
                    }
                }
                const size_t mw_static = (3 * kMwRootMax + kBlock / 64 + 8) * sizeof(double);
                int dev = 0, maxlds = 0;
                const bool attr = hipGetDevice(&dev) == hipSuccess &&
                                  hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess;
                // (with node-node contacts a pair's leader updates its follower's row,
                // which another workgroup's LDS window would hold: vectors in HBM)
                bool lw = one && attr && mw_lds_default() && !D.self_on && need + mw_static <= (size_t)maxlds;
                const size_t wbytes = lw ? (need + 15) / 16 * 16 : 0;
                bool rl = attr && mw_root_lds_default() && rootc > 0 && wbytes + rootc + mw_static <= (size_t)maxlds;
                if ((lw || rl) && configure_mw_lds((size_t)maxlds - mw_static) != hipSuccess)   // the largest any handle may need
                    lw = rl = false;
                if (lw) D.mw_win = upload(s, win);
                s->mw_lw = lw;
                s->mw_lds = lw || rl ? std::max<size_t>(wbytes + (rl ? rootc : 0), 8) : 0;
                D.mw_rootw = upload(s, rootw);
                D.mw_root_lds = rl ? 1 : 0;
                D.mw_root_off = (int)(wbytes / sizeof(double));
                D.mw = W;
                D.mw_root_c0 = rc0;
                D.mw_ptr = upload(s, ptr);
                D.mw_rows = upload(s, mri);
                D.mw_fitems = upload(s, mfi);
                D.mw_bitems = upload(s, mbi);
                D.mw_bgat = upload(s, mgi);
                D.mw_nodes = upload(s, nodes);
                D.mw_sync = (uint32_t *)zeros<double>(s, kMwSyncDoubles);
            }
        }
    }
    D.n_levels = hm.n_levels;
    D.lvl_rows_ptr = upload(s, lrp);
    D.lvl_items_ptr = upload(s, lip);
    D.lvl_team = upload(s, team);
    // the adjoint (one workgroup per handle, no forward to match) keeps the
    // teams the cost model picks for one workgroup
    D.lvl_team_adj = upload(s, team_adj);
    D.lvl_gat_ptr = upload(s, lgp);
    D.lvl_bwd_ptr = upload(s, lbp);
    {   // forward-pass prefetch ranges, by solve phase
        const int L = hm.n_levels;
        std::vector<std::vector<int64_t>> ph(2 * L);
        for (int sn = 0; sn < ns; ++sn) {
            const int l = hm.sup_level[sn], nsz = sns[sn], ld = nsz + snr[sn];
            const int64_t fe = sn + 1 < ns ? goff[sn + 1] : (int64_t)gval.size();
            const int64_t be = sn + 1 < ns ? gofft[sn + 1] : (int64_t)gvalt.size();
            (void)ld;
            (void)nsz;
            ph[l].insert(ph[l].end(), {goff[sn], fe - goff[sn]});
            if (snr[sn] > 0) ph[L + (L - 1 - l)].insert(ph[L + (L - 1 - l)].end(), {gofft[sn], be - gofft[sn]});
        }
        std::vector<int64_t> fpf;
        std::vector<int32_t> fptr(1, 0);
        for (const auto &r : ph) {
            fpf.insert(fpf.end(), r.begin(), r.end());
            fptr.push_back((int32_t)(fpf.size() / 2));
        }
        D.fpf = upload(s, fpf);
        D.fpf_ptr = upload(s, fptr);
        D.fwd_pos = zeros<int64_t>(s, 1);
    }
    D.n_root_rows = (int)root_rows.size();
    D.root_rows = upload(s, root_rows);
    D.bgat = upload(s, bgat);
    D.rows = upload(s, ritems);
    D.fitems = upload(s, fitems);
    D.bitems = upload(s, bitems);
    D.sup_rows = upload(s, rows);
    D.gval = upload(s, gval);
    D.gvalt = upload(s, gvalt);
    D.upd_off = upload(s, uo);
    D.n_ubuf = std::max(uoff[ns], 3);
    // node-centred springs and active curved-bending incidence
    std::vector<int32_t> sp;
    std::vector<SpringInc> sv;
    std::vector<double> srho;
    int nca_bend = 0;
    spring_incidence(hm, order, nca, sp, sv, srho, nca_bend);
    D.sinc_ptr = upload(s, sp);
    D.sinc = upload(s, sv);
    D.sinc_rho = upload(s, srho);
    D.nca_bend = nca_bend;
    std::vector<int32_t> bp(1, 0), bc;
    std::vector<double> bcf;
    for (int i = 0; i < m; ++i) {
        for (auto &pr : inc[i])
            if (pr.first >= nca - nca_bend) { bc.push_back(pr.first); bcf.push_back(pr.second); }
        bp.push_back((int32_t)bc.size());
    }
    D.binc_ptr = upload(s, bp);
    D.binc_con = upload(s, bc);
    D.binc_coef = upload(s, bcf);
    s->factor_bytes = (int64_t)gval.size() * 8;   // per copy (forward and backward each hold one)
    // direct adjoint: its own supernode partition (host model: P's supernodes
    // with merged top separators kept apart, cut into chunks small enough for
    // the register inversion), update lists, scatter targets of A's blocks,
    // solve schedule (built for handles that use the direct adjoint)
    D.adj_direct = hm.adj_solver == SIM_ADJ_DIRECT;
    s->n_ubuf_bwd = D.n_ubuf;
    if (!D.adj_direct) D.ubuf = zeros<double>(s, D.n_ubuf);
    if (D.adj_direct) {
        const int na = (int)hm.lu_c0.size() - 1;
        std::vector<int32_t> ac0(na), an(na), chunk_of(m);
        const std::vector<int32_t> &arptr = hm.lu_R_ptr, &arows = hm.lu_R_rows;
        for (int t = 0; t < na; ++t) {
            ac0[t] = hm.lu_c0[t];
            an[t] = hm.lu_c0[t + 1] - hm.lu_c0[t];
            for (int c = ac0[t]; c < ac0[t] + an[t]; ++c) chunk_of[c] = t;
        }
        std::vector<LuSup> ls(na);
        int64_t off = 0;
        int nmax = 3, ubuf_a = 0;
        for (int t = 0; t < na; ++t) {
            LuSup &q = ls[t];
            q.c0 = ac0[t];
            q.n = an[t];
            q.r = arptr[t + 1] - arptr[t];
            q.rptr = arptr[t];
            q.uoff = ubuf_a;
            ubuf_a += 3 * q.r;
            q.off = off;
            const int64_t N = 3 * (int64_t)q.n, R = 3 * (int64_t)q.r;
            q.ldn = (int32_t)(N + (N & 1));
            q.ldr = (int32_t)(R + (R & 1));
            off += N * q.ldn + N * q.ldr + R * q.ldn;
            nmax = std::max(nmax, (int)N);
        }
        if (nmax > 128) throw std::runtime_error("supernode chunk too large for the direct adjoint");
        // updaters: chunk d reaches chunk t through a run of rows of R_d
        std::vector<std::vector<LuUpd>> ul(na);
        for (int d = 0; d < na; ++d) {
            const int r0 = arptr[d], nr = arptr[d + 1] - arptr[d];
            for (int i = 0; i < nr;) {
                const int t = chunk_of[arows[r0 + i]];
                int j = i;
                while (j < nr && chunk_of[arows[r0 + j]] == t) ++j;
                ul[t].push_back(LuUpd{d, i, j, 0});
                i = j;
            }
        }
        auto pos_in_R = [&](int t, int node) {
            const int *b = arows.data() + arptr[t], *e = arows.data() + arptr[t + 1];
            const int *it = std::lower_bound(b, e, node);
            if (it == e || *it != node) throw std::runtime_error("factor structure misses an entry of A");
            return (int)(it - b);
        };
        // panel rows in t of the rows of R_d from i0 on: nodes of t first, then
        // R_t (every later row of R_d must be a row of R_t); levels: one more
        // than the highest updater
        std::vector<int32_t> up_ptr(1, 0), relmap;
        const std::vector<int32_t> &alevel = hm.lu_level;
        std::vector<LuUpd> upl;
        for (int t = 0; t < na; ++t) {
            for (LuUpd ud : ul[t]) {
                ud.map = (int32_t)relmap.size();
                for (int i = ud.i0; i < arptr[ud.d + 1] - arptr[ud.d]; ++i) {
                    const int node = arows[arptr[ud.d] + i];
                    relmap.push_back(i < ud.i1 ? node - ac0[t] : an[t] + pos_in_R(t, node));
                }
                upl.push_back(ud);
            }
            up_ptr.push_back((int32_t)upl.size());
        }
        const int L = hm.lu_n_levels;
        // scatter target of every block (i, j) of the pattern of K_s (new order).
        // Blocks are stored transposed (column-major): D_t^T (N x N), B_t^T
        // (N x R) and A(t, R_t)^T (R x N), row-major; entry (r, c) of the 3 x 3
        // block (i, j) of A is at kdst + c * kld + r.
        std::vector<int64_t> kdst(kc.size());
        std::vector<int32_t> kld(kc.size());
        for (int i = 0; i < m; ++i) {
            for (int e = kp[i]; e < kp[i + 1]; ++e) {
                const int j = kc[e], ti = chunk_of[i], tj = chunk_of[j];
                if (ti == tj) {
                    const LuSup &q = ls[ti];
                    kdst[e] = q.off + (int64_t)3 * (j - q.c0) * q.ldn + 3 * (i - q.c0);
                    kld[e] = q.ldn;
                } else if (tj < ti) {                   // lower: i in R_tj
                    const LuSup &q = ls[tj];
                    const int64_t N = 3 * (int64_t)q.n;
                    kdst[e] = q.off + N * q.ldn + (int64_t)3 * (j - q.c0) * q.ldr + 3 * pos_in_R(tj, i);
                    kld[e] = q.ldr;
                } else {                                // upper: j in R_ti
                    const LuSup &q = ls[ti];
                    const int64_t N = 3 * (int64_t)q.n;
                    kdst[e] = q.off + N * q.ldn + N * q.ldr + (int64_t)3 * pos_in_R(ti, j) * q.ldn + 3 * (i - q.c0);
                    kld[e] = q.ldn;
                }
            }
        }
        // Delta P blocks: incidence entry (i, c) adds a_ci a_cl G_c to block (i, l)
        std::vector<int32_t> dptr(1, 0), dks;
        for (int i = 0; i < m; ++i) {
            for (int p = ip[i]; p < ip[i + 1]; ++p) {
                const int c = ic[p];
                for (int q = cp[c]; q < cp[c + 1]; ++q) {
                    const int l = cn[q];
                    const int *b = kc.data() + kp[i], *e = kc.data() + kp[i + 1];
                    const int *it = std::lower_bound(b, e, l);
                    if (it == e || *it != l) throw std::runtime_error("K_s pattern misses a constraint coupling");
                    dks.push_back((int32_t)(it - kc.data()));
                }
                dptr.push_back((int32_t)dks.size());
            }
        }
        // solve schedule by level: forward gathers (per node: the update-buffer
        // entries reaching it), backward gathers of x_{R_t}, and the block
        // products in 64-row items (D^{-1}, B, V), balanced over the wavefronts
        std::vector<std::vector<int32_t>> aupd(m);
        for (int d = 0; d < na; ++d)
            for (int q = 0; q < ls[d].r; ++q) aupd[arows[arptr[d] + q]].push_back(ls[d].uoff + 3 * q);
        std::vector<int32_t> aup(1, 0), auo;
        for (int i = 0; i < m; ++i) {
            auo.insert(auo.end(), aupd[i].begin(), aupd[i].end());
            aup.push_back((int32_t)auo.size());
        }
        std::vector<int32_t> lvl(2 * (L + 1), 0);
        std::vector<RowItem> ri;
        std::vector<GatherItem> gat;
        std::vector<std::vector<AdjItem>> phase(3 * L);
        std::vector<std::vector<int64_t>> pf(3 * L);          // blocks read by each phase (prefetch)
        s->lvl_sn.assign(L, {});
        s->lvl_nmax.assign(L, 3);
        for (int l = 0; l < L; ++l) {
            for (int t = 0; t < na; ++t) {
                if (alevel[t] != l) continue;
                const LuSup &q = ls[t];
                const int N = 3 * q.n, R = 3 * q.r, t0 = 3 * q.c0;
                s->lvl_sn[l].push_back(t);
                s->lvl_nmax[l] = std::max(s->lvl_nmax[l], N);
                for (int c = ac0[t]; c < ac0[t] + an[t]; ++c) ri.push_back(RowItem{3 * c, aup[c], aup[c + 1], 0});
                for (int k = 0; k < q.r; ++k) gat.push_back(GatherItem{q.uoff + 3 * k, 3 * arows[q.rptr + k]});
                const int64_t offB = q.off + (int64_t)N * q.ldn, offV = offB + (int64_t)N * q.ldr;
                for (int a = 0; a < N; a += kAdjRows) {  // z_t = D_t^{-1} t_t and x_t = z_t - V_t x_{R_t}
                    const int nr = std::min(kAdjRows, N - a);
                    phase[3 * l].push_back(AdjItem{q.off + a, q.ldn, N, t0, t0 + a, nr, adj_groups(nr, N)});
                    phase[3 * l + 2].push_back(AdjItem{offV + a, q.ldn, R, (int32_t)q.uoff, t0 + a, nr, adj_groups(nr, R)});
                }
                for (int a = 0; a < R; a += kAdjRows) {  // u_t = B_t z_t
                    const int nr = std::min(kAdjRows, R - a);
                    phase[3 * l + 1].push_back(AdjItem{offB + a, q.ldr, N, t0, q.uoff + a, nr, adj_groups(nr, N)});
                }
                pf[3 * l].insert(pf[3 * l].end(), {q.off, (int64_t)N * q.ldn});
                if (R > 0) {
                    pf[3 * l + 1].insert(pf[3 * l + 1].end(), {offB, (int64_t)N * q.ldr});
                    pf[3 * l + 2].insert(pf[3 * l + 2].end(), {offV, (int64_t)R * q.ldn});
                }
            }
            lvl[2 * (l + 1)] = (int32_t)ri.size();
            lvl[2 * (l + 1) + 1] = (int32_t)gat.size();
        }
        std::vector<AdjItem> aitems;
        std::vector<int32_t> aprog, asplit, asptr(1, 0);
        for (const auto &ph : phase) balance_phase(ph, aitems, aprog, asplit, asptr);
        std::vector<int64_t> pfl;
        std::vector<int32_t> pfptr(1, 0);
        for (const auto &r : pf) {
            pfl.insert(pfl.end(), r.begin(), r.end());
            pfptr.push_back((int32_t)(pfl.size() / 2));
        }
        D.ns = na;
        D.lu_nlevels = L;
        D.lu_sup = upload(s, ls);
        D.lu_srows = upload(s, arows);
        D.lu_upd_ptr = upload(s, up_ptr);
        D.lu_upd = upload(s, upl);
        D.lu_relmap = upload(s, relmap);
        D.ks_dst = upload(s, kdst);
        D.ks_ld = upload(s, kld);
        D.dp_ptr = upload(s, dptr);
        D.dp_ks = upload(s, dks);
        D.lu_lvl = upload(s, lvl);
        D.lu_gat = upload(s, gat);
        D.adj_items = upload(s, aitems);
        D.adj_prog = upload(s, aprog);
        D.adj_sptr = upload(s, asptr);
        D.adj_split = upload(s, asplit);
        D.adj_pf = upload(s, pfl);
        D.adj_pfptr = upload(s, pfptr);
        D.adj_pos = zeros<int64_t>(s, 1);
        D.adj_hz = zeros<double>(s, 3 * (size_t)m);
        D.adj_dwc = zeros<double>(s, (size_t)std::max(nca, 1));
        D.lu_rows = upload(s, ri);
        D.lu_upd_off = upload(s, auo);
        D.af_size = off;
        D.af_nmax = nmax;
        // workspace: T blocks (9 m), projection scale + direction (4 nca),
        // |A|_inf (1), perturbed pivots per chunk (na int32)
        D.af_ws_size = 9 * (int64_t)m + 4 * (int64_t)std::max(nca, 1) + 1 + (na + 1) / 2;
        s->n_ubuf_bwd = std::max(D.n_ubuf, ubuf_a);             // the two solves share the update buffer
        D.ubuf = zeros<double>(s, s->n_ubuf_bwd);
    }
    // state and work buffers
    const size_t v3 = 3 * (size_t)m;
    D.x = zeros<double>(s, v3);
    D.v = zeros<double>(s, v3);
    D.vk = zeros<double>(s, v3);
    D.vk1 = zeros<double>(s, v3);
    D.b0 = zeros<double>(s, v3);
    D.rhs = zeros<double>(s, v3);
    D.ysol = zeros<double>(s, v3);
    D.f = zeros<double>(s, v3);
    D.wp = zeros<double>(s, 3 * (size_t)std::max(nca, 1));
    D.mode = zeros<uint8_t>(s, m);
    D.cobst = zeros<int8_t>(s, m);
    D.ubar = zeros<double>(s, v3);
    D.red = zeros<double>(s, 64);
    D.gx = zeros<double>(s, v3);
    D.gv = zeros<double>(s, v3);
    D.zeta = zeros<double>(s, v3);
    D.zeta1 = zeros<double>(s, v3);
    D.zt = zeros<double>(s, v3);
    D.adj_s = zeros<double>(s, std::max(nca, 1));
    D.adj_q = zeros<double>(s, 3 * (size_t)std::max(nca, 1));
    D.adj_pq = zeros<double>(s, 3 * (size_t)std::max(nca, 1));
    D.tblk = zeros<double>(s, 9 * (size_t)m);
    D.dw = zeros<double>(s, std::max(hm.nc, 1));
    D.dmu = zeros<double>(s, kMaxObstacles + 1);
    D.counters = zeros<int64_t>(s, 8);
    D.kry_m = std::min(hm.adj_restart, kKryM);
    D.kry = zeros<double>(s, (size_t)(D.kry_m + 1) * v3);
    // caller-order helpers
    s->d_perm = upload(s, perm);
    std::vector<double> xr(v3);
    for (int i = 0; i < m; ++i)
        for (int d = 0; d < 3; ++d) xr[3 * i + d] = hm.X[3 * perm[i] + d];
    s->rest_x = upload(s, xr);
    s->start_x = zeros<double>(s, v3);
    s->start_v = zeros<double>(s, v3);
    s->d_basew = upload(s, hm.base_w);
    if (!hm.region.empty()) s->d_region = upload(s, hm.region);
    s->d_bend_centers = upload(s, hm.bend_center);
    s->d_modes_tmp = zeros<uint8_t>(s, m);
    if (D.self_on) {
        // node-node contact: caller ids, the nodes sharing a stencil with each
        // node (new order, every spring and bending stencil), search buffers
        D.caller_id = s->d_perm;
        std::vector<std::vector<int32_t>> nb(m);
        for (int c = 0; c < hm.nc; ++c)
            for (int p = hm.c_ptr[c]; p < hm.c_ptr[c + 1]; ++p)
                for (int q = hm.c_ptr[c]; q < hm.c_ptr[c + 1]; ++q)
                    if (p != q) nb[iperm[hm.c_node[p]]].push_back(iperm[hm.c_node[q]]);
        std::vector<int32_t> ap(1, 0), ac;
        for (int i = 0; i < m; ++i) {
            std::sort(nb[i].begin(), nb[i].end());
            nb[i].erase(std::unique(nb[i].begin(), nb[i].end()), nb[i].end());
            ac.insert(ac.end(), nb[i].begin(), nb[i].end());
            ap.push_back((int32_t)ac.size());
        }
        if (ac.empty()) ac.push_back(-1);
        D.adj_ptr = upload(s, ap);
        D.adj_col = upload(s, ac);
        D.ybuf = zeros<double>(s, v3);
        int hs = 1;
        while (hs < 2 * m) hs *= 2;
        D.self_hmask = hs - 1;
        D.self_inv_cell = 1.0 / (hm.self_r * (1.0 + 1e-6));
        D.self_head = zeros<int32_t>(s, hs);
        D.self_next = zeros<int32_t>(s, m);
        D.cand = zeros<int32_t>(s, m);
        D.partner = zeros<int32_t>(s, m);
    }
    s->dd = (SimDev *)dev_alloc(s, sizeof(SimDev));
    // LDS placement: the solve vectors first, then the update buffer, then x_n
    int dev = 0, maxlds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        throw std::runtime_error("hip attribute");
    if (kernel_static_lds(&s->static_fwd, &s->static_bwd) != hipSuccess) throw std::runtime_error("hip attribute");
    if (hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        throw std::runtime_error("hip attribute");
    s->max_lds = (size_t)maxlds;
    if (configure_lds(s->max_lds - s->static_fwd, s->max_lds - s->static_bwd) != hipSuccess) s->max_lds = 0;
    plan_lds(s, s->flags_fwd, s->lds_fwd, true);
    plan_lds(s, s->flags_bwd, s->lds_bwd, false);
}

// A batched launch shares one placement: the same greedy choice as for one
// handle (vectors, then update buffer, then positions), each kind added when it
// fits every handle of the launch.  (Intersecting the handles' own choices can
// leave nothing: a large handle without vectors in LDS and a middle one
// without positions.)
size_t batch_lds(sim *const *sims, int n, bool fwd, int &flags) {
    auto fits = [&](int f, size_t &mx) {
        mx = 0;
        for (int i = 0; i < n; ++i) {
            const size_t st = fwd ? sims[i]->static_fwd : sims[i]->static_bwd;
            const size_t avail = sims[i]->max_lds > st ? sims[i]->max_lds - st : 0;
            const size_t b = lds_bytes(sims[i], f, fwd);
            mx = std::max(mx, b);
            if (b > avail) return false;
        }
        return true;
    };
    flags = 0;
    size_t bytes = 0, mx = 0;
    const int allowed = lds_allowed();
    for (int bit : {kLdsVectors, kLdsUpdates, kLdsPositions}) {
        if ((!fwd && bit == kLdsPositions) || !(allowed & bit)) continue;
        if (fits(flags | bit, mx)) {
            flags |= bit;
            bytes = mx;
        }
    }
    return bytes;
}

int push_desc(sim *s) {
    return hip_err(hipMemcpyAsync(s->dd, &s->hd, sizeof(SimDev), hipMemcpyHostToDevice, s->stream));
}

// make room for `cap` step records
int fac_idle(sim *s);

void ensure_records(sim *s, int cap) {
    if (s->hd.rec_cap >= cap && s->hd.rec_x) return;
    if (fac_idle(s)) throw std::runtime_error("hip");
    dev_release(s, s->hd.rec_x);
    dev_release(s, s->hd.rec_v);
    dev_release(s, s->hd.rec_ubar);
    dev_release(s, s->hd.rec_mode);
    dev_release(s, s->hd.rec_obst);
    dev_release(s, s->hd.rec_partner);
    s->hd.rec_partner = nullptr;
    const size_t v3 = 3 * (size_t)s->hd.m;
    s->hd.rec_x = (double *)dev_alloc(s, (cap + 1) * v3 * sizeof(double));
    s->hd.rec_v = (double *)dev_alloc(s, (cap + 1) * v3 * sizeof(double));
    s->hd.rec_ubar = (double *)dev_alloc(s, cap * v3 * sizeof(double));
    s->hd.rec_mode = (uint8_t *)dev_alloc(s, (size_t)cap * s->hd.m);
    s->hd.rec_obst = (int8_t *)dev_alloc(s, (size_t)cap * s->hd.m);
    if (s->hd.self_on) s->hd.rec_partner = (int32_t *)dev_alloc(s, (size_t)cap * s->hd.m * sizeof(int32_t));
    s->hd.rec_cap = cap;
}

// room for `cap` step factors of the direct adjoint
void ensure_af(sim *s, int cap) {
    if (s->af_cap >= cap && s->hd.af) return;
    if (fac_idle(s)) throw std::runtime_error("hip");
    dev_release(s, s->hd.af);
    dev_release(s, s->hd.af_ws);
    s->hd.af = nullptr;
    s->hd.af_ws = nullptr;
    s->af_cap = 0;
    s->hd.af = (double *)dev_alloc(s, (size_t)cap * s->hd.af_size * sizeof(double));
    s->hd.af_ws = (double *)dev_alloc(s, (size_t)cap * s->hd.af_ws_size * sizeof(double));
    s->af_cap = cap;
}

int copy_d2d(sim *s, void *dst, const void *src, size_t bytes) {
    return hip_err(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s->stream));
}

int seg_len(const sim *s) { return s->hm.checkpoint_every > 0 ? s->hm.checkpoint_every : 0; }

// Waits for the overlapped factorisation (before its buffers are released or
// its factors are replaced) and forgets it.
int fac_idle(sim *s) {
    s->prefactored = 0;
    return s->fac_stream ? hip_err(hipStreamSynchronize(s->fac_stream)) : SIM_OK;
}

// Forward chunks (end steps) when the factorisation overlaps the forward pass
// (empty: no overlap).  Each chunk is half the steps left, down to 8: the
// factorisation of a chunk (≈ 1/10 of its forward time) hides under the
// next one, and only the last, short chunk's is left for the backward pass.
std::vector<int> overlap_chunks(const sim *s, int n_steps) {
    std::vector<int> ends;
    if (!s->hd.adj_direct || seg_len(s) > 0 || s->hm.adj_window > 0 || n_steps < 16) return ends;
    const char *e = std::getenv("DIFFCLOTH_FACTOR_OVERLAP");
    if (e && std::atoi(e) == 0) return ends;
    int a = 0;
    while (n_steps - a > 8) {
        a += std::max(4, (n_steps - a) / 2);
        ends.push_back(a);
    }
    if (a < n_steps) ends.push_back(n_steps);
    return ends;
}

// Forward over [a, b) from the handle's current state into the record buffer.
// Forward launch of one handle (descriptor already pushed): the
// multi-workgroup kernel when the handle's tree allows it, its barrier block
// cleared first (a fill kernel), else one workgroup (plus prefetchers).
int launch_single_forward(sim *s) {
    if (s->hd.mw >= 2) {
        int rc = hip_err(launch_fill((double *)s->hd.mw_sync, 0.0, kMwSyncDoubles, s->stream));
        if (!rc)
            rc = hip_err(launch_forward_mw(s->dd, s->hd.mw, s->hd.mixed != 0, has_mesh(&s, 1), s->mw_lw, s->mw_lds,
                                           mw_threads_default(), s->stream));
        s->mw_used = true;
        return rc;
    }
    return hip_err(launch_forward(s->dd, 1, s->hd.mixed != 0, s->lds_fwd, s->flags_fwd, fwd_helpers(&s, 1),
                                  has_mesh(&s, 1), s->stream));
}

int run_forward_range(sim *s, int a, int b) {
    s->hd.step_begin = a;
    s->hd.step_end = b;
    s->hd.rec_step0 = a;
    ++s->hd.fwd_epoch;
    int rc = push_desc(s);
    if (rc) return rc;
    return launch_single_forward(s);
}

// A multi-workgroup forward launch since the last check gave up at a barrier
// (a workgroup waited longer than mw_spin): SIM_ESYNC; clears the flag.
int mw_check(sim *s) {
    if (!s->mw_used) return SIM_OK;
    uint32_t flag[4] = {0, 0, 0, 0};
    int rc = hip_err(hipMemcpyAsync(flag, s->hd.mw_sync, sizeof(flag), hipMemcpyDeviceToHost, s->stream));
    if (!rc) rc = hip_err(hipStreamSynchronize(s->stream));
    if (rc) return rc;
    s->mw_used = false;
    return flag[2] ? SIM_ESYNC : SIM_OK;
}

// Timing event k of the handle's stream (0/1 forward start/end, 2/3 backward).
int time_mark(sim *s, int k) {
    if (!s->tev[k]) {
        const int rc = hip_err(hipEventCreate(&s->tev[k]));
        if (rc) return rc;
    }
    return hip_err(hipEventRecord(s->tev[k], s->stream));
}

int read_counters(sim *s) {
    int rc = hip_err(hipMemcpyAsync(s->counters_host, s->hd.counters, sizeof(s->counters_host), hipMemcpyDeviceToHost,
                                    s->stream));
    if (rc) return rc;
    return hip_err(hipStreamSynchronize(s->stream));
}

template <class F>
int guarded(F &&f) {
    try {
        return f();
    } catch (const std::bad_alloc &) {
        return SIM_ENOMEM;
    } catch (...) {
        return SIM_EHIP;
    }
}

}  // namespace

extern "C" {

struct sim_plan {
    HostModel hm;
};

int sim_plan_create(const sim_mesh_t *mesh, const sim_params_t *params, sim_plan_t **out) {
    if (!out) return SIM_EINVAL;
    *out = nullptr;
    sim_plan *pl = new (std::nothrow) sim_plan();
    if (!pl) return SIM_ENOMEM;
    // the host build allocates (std::map, std::vector): no exception may leave the ABI
    int rc = guarded([&] { return pl->hm.build(mesh, params); });
    if (rc == SIM_OK) rc = guarded([&] { return pl->hm.order_and_factor(leaf_size_default(mesh->n_nodes), merge_cap_default()); });
    if (rc != SIM_OK) {
        delete pl;
        return rc;
    }
    *out = pl;
    return SIM_OK;
}

void sim_plan_destroy(sim_plan_t *plan) { delete plan; }

int sim_create_from_plan(sim_plan_t *plan, void *hip_stream, sim_alloc_fn alloc, sim_free_fn free_fn,
                         void *alloc_ctx, sim_t **out) {
    if (!out || !plan) return SIM_EINVAL;
    *out = nullptr;
    sim *s = new (std::nothrow) sim();
    if (!s) return SIM_ENOMEM;
    s->stream = (hipStream_t)hip_stream;
    s->alloc = alloc;
    s->free_fn = free_fn;
    s->ctx = alloc_ctx;
    s->hm = std::move(plan->hm);
    // the device set-up queries and sets kernel attributes (which loads the
    // code object on first use) and uploads the tables: one handle at a time
    // in a process
    static std::mutex device_setup;
    std::lock_guard<std::mutex> lock(device_setup);
    int rc = guarded([&] {
        build_device(s);
        int r = push_desc(s);
        if (r) return r;
        // device address of the allocation-free forward's scratch, taken once
        // per device at set-up (a failure surfaces when that entry point is called)
        void *scratch_addr = nullptr;
        (void)noalloc_scratch(&scratch_addr);
        r = sim_set_state(s, nullptr, nullptr);
        if (r) return r;
        return hip_err(hipStreamSynchronize(s->stream));
    });
    if (rc != SIM_OK) {
        plan->hm = std::move(s->hm);        // the plan stays usable
        sim_destroy(s);
        return rc;
    }
    delete plan;
    *out = s;
    return SIM_OK;
}

int sim_create(const sim_mesh_t *mesh, const sim_params_t *params, void *hip_stream, sim_alloc_fn alloc,
               sim_free_fn free_fn, void *alloc_ctx, sim_t **out) {
    if (!out) return SIM_EINVAL;
    *out = nullptr;
    sim_plan_t *plan = nullptr;
    int rc = sim_plan_create(mesh, params, &plan);
    if (rc != SIM_OK) return rc;
    rc = sim_create_from_plan(plan, hip_stream, alloc, free_fn, alloc_ctx, out);
    if (rc != SIM_OK) sim_plan_destroy(plan);
    return rc;
}

int sim_set_state(sim_t *s, const double *x0_dev, const double *v0_dev) {
    if (!s) return SIM_EINVAL;
    const int m = s->hd.m;
    const size_t v3b = 3 * (size_t)m * sizeof(double);
    int rc;
    if (x0_dev) rc = hip_err(launch_permute3(x0_dev, s->start_x, s->d_perm, m, false, s->stream));
    else rc = copy_d2d(s, s->start_x, s->rest_x, v3b);
    if (rc) return rc;
    if (v0_dev) rc = hip_err(launch_permute3(v0_dev, s->start_v, s->d_perm, m, false, s->stream));
    else rc = hip_err(launch_fill(s->start_v, 0.0, 3 * (int64_t)m, s->stream));
    if (rc) return rc;
    s->T = -1;
    s->phase = 0;
    s->prefactored = 0;
    return SIM_OK;
}


int sim_set_external_force(sim_t *s, const double *force_dev, int32_t n_scale, const double *scale_host) {
    if (!s) return SIM_EINVAL;
    if (force_dev && scale_host) {
        if (n_scale < 1) return SIM_EINVAL;
        for (int n = 0; n < n_scale; ++n)
            if (!std::isfinite(scale_host[n])) return SIM_EINVAL;
    }
    return guarded([&] {
        int rc = hip_err(hipStreamSynchronize(s->stream));   // no pass still reads the old force
        if (rc) return rc;
        s->T = -1;
        s->phase = 0;
        s->prefactored = 0;
        if (!force_dev) {
            s->hd.fext = nullptr;
            s->hd.fscale = nullptr;
            s->n_fscale = 0;
            return SIM_OK;
        }
        const int m = s->hd.m;
        if (!s->fext_buf) s->fext_buf = (double *)dev_alloc(s, 3 * (size_t)m * sizeof(double));
        rc = hip_err(launch_permute3(force_dev, s->fext_buf, s->d_perm, m, false, s->stream));
        if (rc) return rc;
        s->hd.fext = s->fext_buf;
        s->hd.fscale = nullptr;
        s->n_fscale = 0;
        if (scale_host) {
            if (s->fscale_cap < n_scale) {
                dev_release(s, s->fscale_buf);
                s->fscale_buf = nullptr;
                s->fscale_cap = 0;
                s->fscale_buf = (double *)dev_alloc(s, n_scale * sizeof(double));
                s->fscale_cap = n_scale;
            }
            rc = hip_err(hipMemcpyAsync(s->fscale_buf, scale_host, n_scale * sizeof(double), hipMemcpyHostToDevice,
                                        s->stream));
            if (!rc) rc = hip_err(hipStreamSynchronize(s->stream));   // scale_host may go away on return
            if (rc) return rc;
            s->hd.fscale = s->fscale_buf;
            s->n_fscale = n_scale;
        }
        return SIM_OK;
    });
}

int sim_set_material(sim_t *s, const double *edge_stiffness, const double *bend_weight, const double *region_scale,
                     const double *obstacle_mu) {
    if (!s) return SIM_EINVAL;
    const HostModel &hm = s->hm;
    auto bad = [](double v) { return !std::isfinite(v); };
    if (edge_stiffness)
        for (int e = 0; e < hm.n_edges; ++e) {
            if (bad(edge_stiffness[e])) return SIM_ENONFINITE;
            if (edge_stiffness[e] < 0) return SIM_EINVAL;
        }
    if (bend_weight) {
        if (bad(*bend_weight)) return SIM_ENONFINITE;
        if (*bend_weight < 0) return SIM_EINVAL;
    }
    if (region_scale) {
        if (hm.region_scale.empty()) return SIM_EINVAL;
        for (size_t r = 0; r < hm.region_scale.size(); ++r) {
            if (bad(region_scale[r])) return SIM_ENONFINITE;
            if (region_scale[r] < 0) return SIM_EINVAL;
        }
    }
    if (obstacle_mu)
        for (size_t o = 0; o < hm.obstacles.size(); ++o) {
            if (bad(obstacle_mu[o])) return SIM_ENONFINITE;
            if (obstacle_mu[o] < 0) return SIM_EINVAL;
        }
    return guarded([&] {
        HostModel nm = hm;                        // the handle keeps its material until all succeeded
        if (edge_stiffness)
            for (int e = 0; e < nm.n_edges; ++e) nm.base_w[e] = edge_stiffness[e];
        if (bend_weight)
            for (int b = 0; b < nm.n_bend; ++b) nm.base_w[nm.n_edges + b] = *bend_weight;
        if (region_scale) nm.region_scale.assign(region_scale, region_scale + nm.region_scale.size());
        if (obstacle_mu)
            for (size_t o = 0; o < nm.obstacles.size(); ++o) nm.obstacles[o].mu = obstacle_mu[o];
        const bool refactor = edge_stiffness || bend_weight || region_scale;
        SimDev &D = s->hd;
        std::vector<int32_t> kp, kc, sp;
        std::vector<double> kv, cw, gval, gvalt;
        std::vector<float> kvf, cwf;
        std::vector<int64_t> goff, gofft;
        std::vector<SpringInc> sv;
        int rc = fac_idle(s);                    // the overlapped factorisation reads these tables
        if (rc) return rc;
        if (refactor) {
            nm.apply_regions();
            rc = nm.assemble_ks(true);
            if (!rc) rc = nm.factor();
            if (rc) return rc;
            ks_new_order(nm, kp, kc, kv, kvf);
            slot_weights(nm, s->corder, cw, cwf);
            int nca_bend = 0;
            std::vector<double> srho;
            spring_incidence(nm, s->corder, s->nca, sp, sv, srho, nca_bend);
            stacked_factor(nm, gval, gvalt, goff, gofft);
            auto put = [&](const void *dst, const void *src, size_t bytes) {
                if (!rc && bytes)
                    rc = hip_err(hipMemcpyAsync(const_cast<void *>(dst), src, bytes, hipMemcpyHostToDevice, s->stream));
            };
            put(D.ks_val, kv.data(), kv.size() * sizeof(double));
            put(D.ks_valf, kvf.data(), kvf.size() * sizeof(float));
            put(D.c_w, cw.data(), cw.size() * sizeof(double));
            put(D.c_wf, cwf.data(), cwf.size() * sizeof(float));
            put(D.sinc, sv.data(), sv.size() * sizeof(SpringInc));
            put(D.sinc_rho, srho.data(), srho.size() * sizeof(double));
            put(D.gval, gval.data(), gval.size() * sizeof(double));
            put(D.gvalt, gvalt.data(), gvalt.size() * sizeof(double));
            put(s->d_basew, nm.base_w.data(), nm.base_w.size() * sizeof(double));
        }
        if (!rc) {
            for (size_t o = 0; o < nm.obstacles.size(); ++o) D.obst[o].mu = nm.obstacles[o].mu;
            rc = push_desc(s);
        }
        const int rs = hip_err(hipStreamSynchronize(s->stream));    // host staging buffers end here
        if (!rc) rc = rs;
        if (rc) return rc;
        s->hm = std::move(nm);
        s->T = -1;
        s->phase = 0;
        return SIM_OK;
    });
}

namespace {

// Prepare a handle for a forward pass of n_steps (records / checkpoints) and reset its state.
int prepare_forward(sim *s, int n_steps) {
    if (s->hd.fscale && n_steps > s->n_fscale) return SIM_EINVAL;   // multipliers run out
    if (fac_idle(s)) return SIM_EHIP;        // the records are about to be overwritten
    const int k = seg_len(s);
    const int cap = k > 0 ? std::min(k, n_steps) : n_steps;
    ensure_records(s, std::max(cap, 1));
    if (s->step_info_cap < n_steps) {
        dev_release(s, s->hd.step_info);
        s->hd.step_info = nullptr;
        s->step_info_cap = 0;
        s->hd.step_info = (int32_t *)dev_alloc(s, 4 * (size_t)n_steps * sizeof(int32_t));
        s->step_info_cap = n_steps;
    }
    const size_t v3b = 3 * (size_t)s->hd.m * sizeof(double);
    if (k > 0) {
        const int nseg = (n_steps + k - 1) / k;
        if (s->ckpt_cap < nseg) {
            dev_release(s, s->ckpt);
            s->ckpt = (double *)dev_alloc(s, (size_t)nseg * 3 * v3b);
            s->ckpt_cap = nseg;
        }
    }
    int rc = copy_d2d(s, s->hd.x, s->start_x, v3b);
    if (!rc) rc = copy_d2d(s, s->hd.v, s->start_v, v3b);
    if (!rc) rc = hip_err(launch_fill(s->hd.f, 0.0, 3 * (int64_t)s->hd.m, s->stream));   // no impulses before step 0
    if (!rc) rc = hip_err(hipMemsetAsync(s->hd.counters, 0, 8 * sizeof(int64_t), s->stream));
    return rc;
}

// Checkpoint seg: the state entering its first step and the contact impulses
// of the step before (the warm start of that step).
int save_ckpt(sim *s, int seg) {
    const size_t v3 = 3 * (size_t)s->hd.m, b = v3 * sizeof(double);
    double *c = s->ckpt + (size_t)seg * 3 * v3;
    int rc = copy_d2d(s, c, s->hd.x, b);
    if (!rc) rc = copy_d2d(s, c + v3, s->hd.v, b);
    if (!rc) rc = copy_d2d(s, c + 2 * v3, s->hd.f, b);
    return rc;
}

int load_ckpt(sim *s, int seg) {
    const size_t v3 = 3 * (size_t)s->hd.m, b = v3 * sizeof(double);
    const double *c = s->ckpt + (size_t)seg * 3 * v3;
    int rc = copy_d2d(s, s->hd.x, c, b);
    if (!rc) rc = copy_d2d(s, s->hd.v, c + v3, b);
    if (!rc) rc = copy_d2d(s, s->hd.f, c + 2 * v3, b);
    return rc;
}

int factor_pairs(sim *owner, const SimDev *d_descs, const std::vector<sim *> &hs, const std::vector<int32_t> &pairs,
                 hipStream_t st);

// Forward pass in chunks (ending at ends[]) on the handle's stream; after each chunk
// a second stream factors the chunk's steps (their records are complete once
// the chunk has run), so only the last chunk's factorisation is left for the
// backward pass.  Results are those of one launch (the kernel keeps no state
// in LDS across steps).
int forward_overlapped(sim *s, int n_steps, const std::vector<int> &ends) {
    int rc = fac_idle(s);
    if (rc) return rc;
    if (!s->fac_stream) {
        rc = hip_err(hipStreamCreateWithFlags(&s->fac_stream, hipStreamNonBlocking));
        if (!rc) rc = hip_err(hipEventCreateWithFlags(&s->fac_ev, hipEventDisableTiming));
        if (!rc) rc = hip_err(hipEventCreateWithFlags(&s->fac_done, hipEventDisableTiming));
        if (!rc && !s->dd_fac) s->dd_fac = (SimDev *)dev_alloc(s, sizeof(SimDev));
        if (rc) return rc;
    }
    ensure_af(s, n_steps);
    {   // work buffer for the largest chunk, sized before any factorisation runs
        int ch = ends[0];
        for (size_t c = 1; c < ends.size(); ++c) ch = std::max(ch, ends[c] - ends[c - 1]);
        size_t need = 2 * (size_t)ch;
        for (const auto &l : s->lvl_sn) need += 3 * l.size() * (size_t)ch;
        if (s->work_cap < need) {
            dev_release(s, s->d_work);
            s->d_work = (int32_t *)dev_alloc(s, need * sizeof(int32_t));
            s->work_cap = need;
        }
    }
    s->hd_fac = s->hd;                       // factor descriptor: slot k = step k, records from step 0
    s->hd_fac.af_step0 = 0;
    s->hd_fac.rec_step0 = 0;
    rc = hip_err(hipMemcpyAsync(s->dd_fac, &s->hd_fac, sizeof(SimDev), hipMemcpyHostToDevice, s->stream));
    int pa = -1, pb = -1;                    // chunk whose factorisation is still to be queued
    for (size_t c = 0; c < ends.size() && !rc; ++c) {
        const int a = c ? ends[c - 1] : 0, b = ends[c];
        s->hd.step_begin = a;
        s->hd.step_end = b;
        s->hd.rec_step0 = 0;
        ++s->hd.fwd_epoch;
        rc = push_desc(s);
        if (!rc) rc = launch_single_forward(s);
        if (!rc && pa >= 0) {                // the previous chunk, queued behind this one's launch
            std::vector<int32_t> pairs;
            for (int n = pa; n < pb; ++n) { pairs.push_back(0); pairs.push_back(n); }
            rc = factor_pairs(s, s->dd_fac, {s}, pairs, s->fac_stream);
        }
        if (!rc) rc = hip_err(hipEventRecord(s->fac_ev, s->stream));
        if (!rc) rc = hip_err(hipStreamWaitEvent(s->fac_stream, s->fac_ev, 0));
        pa = a;
        pb = b;
    }
    if (!rc && pa >= 0) {
        std::vector<int32_t> pairs;
        for (int n = pa; n < pb; ++n) { pairs.push_back(0); pairs.push_back(n); }
        rc = factor_pairs(s, s->dd_fac, {s}, pairs, s->fac_stream);
    }
    if (!rc) rc = hip_err(hipEventRecord(s->fac_done, s->fac_stream));
    if (!rc) s->prefactored = n_steps;
    return rc;
}

// Forward pass; with checkpointing, segment by segment (state saved at each segment start).
int forward_all(sim *s, int n_steps, double *x_traj_dev) {
    const int m = s->hd.m;
    const size_t v3 = 3 * (size_t)m;
    const int k = seg_len(s);
    int rc = SIM_OK;
    if (k <= 0) {
        const std::vector<int> ends = overlap_chunks(s, n_steps);
        s->fwd_launches = ends.empty() ? 1 : (int)ends.size();
        if (!ends.empty()) rc = forward_overlapped(s, n_steps, ends);
        else rc = run_forward_range(s, 0, n_steps);
        if (!rc && x_traj_dev)
            for (int n = 0; n <= n_steps && !rc; ++n)
                rc = hip_err(launch_permute3(s->hd.rec_x + n * v3, x_traj_dev + n * v3, s->d_perm, m, true, s->stream));
        return rc;
    }
    s->fwd_launches = (n_steps + k - 1) / k;
    for (int a = 0, seg = 0; a < n_steps && !rc; a += k, ++seg) {
        const int b = std::min(n_steps, a + k);
        rc = save_ckpt(s, seg);
        if (!rc) rc = run_forward_range(s, a, b);
        if (!rc && x_traj_dev)
            for (int n = a; n <= b && !rc; ++n)
                rc = hip_err(launch_permute3(s->hd.rec_x + (n - a) * v3, x_traj_dev + n * v3, s->d_perm, m, true,
                                             s->stream));
    }
    return rc;
}

int finish_forward(sim *s, int n_steps, double *xT_dev, double *vT_dev) {
    const int m = s->hd.m;
    int rc = mw_check(s);
    if (rc) s->T = -1;                        // nothing usable was recorded
    if (!rc && xT_dev) rc = hip_err(launch_permute3(s->hd.x, xT_dev, s->d_perm, m, true, s->stream));
    if (!rc && vT_dev) rc = hip_err(launch_permute3(s->hd.v, vT_dev, s->d_perm, m, true, s->stream));
    if (!rc) rc = read_counters(s);
    if (!rc) {
        s->T = n_steps;
        s->phase = 2;
    }
    return rc;
}

// Zero the parameter-gradient accumulators of a backward pass over the T
// recorded steps (weights, friction, external force).
int zero_param_grads(sim *s) {
    int rc = hip_err(launch_fill(s->hd.dw, 0.0, std::max(s->hm.nc, 1), s->stream));
    if (!rc) rc = hip_err(launch_fill(s->hd.dmu, 0.0, kMaxObstacles + 1, s->stream));
    if (!rc && s->hd.fext) {
        if (!s->dfext_buf) s->dfext_buf = (double *)dev_alloc(s, 3 * (size_t)s->hd.m * sizeof(double));
        if (s->dfscale_cap < std::max(s->T, 1)) {
            dev_release(s, s->dfscale_buf);
            s->dfscale_buf = nullptr;
            s->dfscale_cap = 0;
            s->dfscale_buf = (double *)dev_alloc(s, std::max(s->T, 1) * sizeof(double));
            s->dfscale_cap = std::max(s->T, 1);
        }
        s->hd.dfext = s->dfext_buf;
        s->hd.dfscale = s->dfscale_buf;
        rc = hip_err(launch_fill(s->hd.dfext, 0.0, 3 * (int64_t)s->hd.m, s->stream));
        if (!rc) rc = hip_err(launch_fill(s->hd.dfscale, 0.0, s->dfscale_cap, s->stream));
    }
    return rc;
}

// Seed the adjoint: gx = dL/dx_T (+ per-step term at T), gv = dL/dv_T; zero the accumulators.
int prepare_backward(sim *s, const double *dL_dxT, const double *dL_dvT, const double *dL_dx_steps) {
    const int m = s->hd.m, T = s->T;
    const size_t v3 = 3 * (size_t)m;
    int rc = SIM_OK;
    if (dL_dx_steps) {
        if (s->gsteps_cap < T + 1) {
            dev_release(s, s->gsteps);
            s->gsteps = (double *)dev_alloc(s, (T + 1) * v3 * sizeof(double));
            s->gsteps_cap = T + 1;
        }
        for (int n = 0; n <= T && !rc; ++n)
            rc = hip_err(launch_permute3(dL_dx_steps + n * v3, s->gsteps + n * v3, s->d_perm, m, false, s->stream));
        s->hd.gx_steps = s->gsteps;
    } else {
        s->hd.gx_steps = nullptr;
    }
    if (rc) return rc;
    if (dL_dxT) rc = hip_err(launch_permute3(dL_dxT, s->hd.gx, s->d_perm, m, false, s->stream));
    else rc = hip_err(launch_fill(s->hd.gx, 0.0, (int64_t)v3, s->stream));
    if (!rc && dL_dx_steps) {
        // gx += per-step term at T (done on the host side of the stream: tiny)
        std::vector<double> a(v3), b(v3);
        rc = hip_err(hipMemcpyAsync(a.data(), s->hd.gx, v3 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        if (!rc) rc = hip_err(hipMemcpyAsync(b.data(), s->gsteps + T * v3, v3 * sizeof(double), hipMemcpyDeviceToHost,
                                             s->stream));
        if (!rc) rc = hip_err(hipStreamSynchronize(s->stream));
        for (size_t i = 0; i < v3 && !rc; ++i) a[i] += b[i];
        if (!rc) rc = hip_err(hipMemcpyAsync(s->hd.gx, a.data(), v3 * sizeof(double), hipMemcpyHostToDevice, s->stream));
        if (!rc) rc = hip_err(hipStreamSynchronize(s->stream));
    }
    if (!rc) {
        if (dL_dvT) rc = hip_err(launch_permute3(dL_dvT, s->hd.gv, s->d_perm, m, false, s->stream));
        else rc = hip_err(launch_fill(s->hd.gv, 0.0, (int64_t)v3, s->stream));
    }
    if (!rc) rc = zero_param_grads(s);
    if (!rc) rc = hip_err(hipMemsetAsync(s->hd.counters, 0, 8 * sizeof(int64_t), s->stream));
    return rc;
}

// Direct adjoint factorisation of the (handle, slot) pairs listed in `pairs`
// (handle = index into hs and into the device descriptor array d_descs): one
// assembly launch, then one launch per elimination level with a workgroup per
// (handle, slot, supernode).  The work lists go through owner's buffers; the
// previous use of them is waited for first.
int factor_pairs(sim *owner, const SimDev *d_descs, const std::vector<sim *> &hs, const std::vector<int32_t> &pairs,
                 hipStream_t st) {
    if (pairs.empty()) return SIM_OK;
    int rc = hip_err(hipStreamSynchronize(st));
    if (rc) return rc;
    int L = 0;
    for (sim *h : hs) L = std::max(L, (int)h->lvl_sn.size());
    std::vector<int> nmax(L, 3);
    for (size_t p = 0; p < pairs.size(); p += 2) {
        const sim *h = hs[pairs[p]];
        for (size_t l = 0; l < h->lvl_nmax.size(); ++l) nmax[l] = std::max(nmax[l], h->lvl_nmax[l]);
    }
    std::vector<int32_t> &buf = owner->h_work;
    buf = pairs;
    std::vector<size_t> loff(L + 1);
    for (int l = 0; l < L; ++l) {
        loff[l] = buf.size();
        for (size_t p = 0; p < pairs.size(); p += 2) {
            const sim *h = hs[pairs[p]];
            if (l >= (int)h->lvl_sn.size()) continue;
            for (int sn : h->lvl_sn[l]) {
                buf.push_back(pairs[p]);
                buf.push_back(pairs[p + 1]);
                buf.push_back(sn);
            }
        }
    }
    loff[L] = buf.size();
    if (owner->work_cap < buf.size()) {
        dev_release(owner, owner->d_work);
        owner->d_work = nullptr;
        owner->work_cap = 0;
        owner->d_work = (int32_t *)dev_alloc(owner, buf.size() * sizeof(int32_t));
        owner->work_cap = buf.size();
    }
    rc = hip_err(hipMemcpyAsync(owner->d_work, buf.data(), buf.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    if (!rc) rc = hip_err(launch_adj_assemble(d_descs, owner->d_work, (int)pairs.size() / 2, st));
    for (int l = 0; l < L && !rc; ++l)
        rc = hip_err(launch_adj_factor_level(d_descs, owner->d_work + loff[l], (int)((loff[l + 1] - loff[l]) / 3),
                                             nmax[l], st));
    return rc;
}

// Direct adjoint: factor steps [a, b) of one handle (records in place, rec_step0 set).
int factor_steps(sim *s, int a, int b) {
    if (!s->hd.adj_direct) return SIM_OK;
    if (a == 0 && s->prefactored > 0 && b == s->prefactored) {  // factored during the forward pass
        s->hd.af_step0 = 0;
        return hip_err(hipStreamWaitEvent(s->stream, s->fac_done, 0));
    }
    int rc0 = fac_idle(s);                   // these slots are about to be overwritten
    if (rc0) return rc0;
    ensure_af(s, b - a);
    s->hd.af_step0 = a;
    int rc = push_desc(s);
    if (rc) return rc;
    std::vector<int32_t> pairs;
    for (int k = 0; k < b - a; ++k) { pairs.push_back(0); pairs.push_back(k); }
    return factor_pairs(s, s->dd, {s}, pairs, s->stream);
}

// Backward over recorded steps [a, b) (records from rec_step0 on): with the
// direct adjoint in windows of adj_window steps, each factored just before its
// solves (the last window first).
int backward_range(sim *s, int a, int b) {
    const int W = s->hd.adj_direct && s->hm.adj_window > 0 ? s->hm.adj_window : b - a;
    for (int hi = b; hi > a;) {
        const int lo = std::max(a, hi - W);
        s->hd.step_begin = lo;
        s->hd.step_end = hi;
        ++s->hd.adj_epoch;                                   // tags this launch's published positions
        int rc = factor_steps(s, lo, hi);
        if (!rc) rc = push_desc(s);
        if (!rc)
            rc = hip_err(launch_backward(s->dd, 1, s->hd.mixed != 0, s->lds_bwd, bwd_variant(s, s->flags_bwd),
                                         s->hd.adj_direct ? adj_helpers_default() : 0, has_mesh(&s, 1), s->stream));
        if (rc) return rc;
        hi = lo;
    }
    return SIM_OK;
}

int backward_all(sim *s) {
    const int T = s->T, k = seg_len(s);
    const size_t v3 = 3 * (size_t)s->hd.m;
    if (k <= 0) {
        s->hd.rec_step0 = 0;
        return backward_range(s, 0, T);
    }
    const int nseg = (T + k - 1) / k;
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int a = seg * k, b = std::min(T, a + k);
        int rc = load_ckpt(s, seg);
        if (!rc) rc = run_forward_range(s, a, b);             // recompute the segment's records
        if (rc) return rc;
        s->hd.rec_step0 = a;
        rc = backward_range(s, a, b);
        if (rc) return rc;
    }
    return SIM_OK;
}

int write_grads(sim *s, const sim_grads_t *out) {
    const int m = s->hd.m;
    int rc = SIM_OK;
    if (!out) return rc;
    if (out->dx0) rc = hip_err(launch_permute3(s->hd.gx, out->dx0, s->d_perm, m, true, s->stream));
    if (!rc && out->dv0) rc = hip_err(launch_permute3(s->hd.gv, out->dv0, s->d_perm, m, true, s->stream));
    if (!rc && out->dw_edge && s->hm.n_edges)
        rc = copy_d2d(s, out->dw_edge, s->hd.dw, s->hm.n_edges * sizeof(double));
    if (!rc && out->dw_bend) {
        rc = hip_err(launch_fill(out->dw_bend, 0.0, m, s->stream));
        if (!rc)
            rc = hip_err(launch_scatter_bend(s->hd.dw, s->d_bend_centers, s->hm.n_edges, s->hm.n_bend, out->dw_bend,
                                             s->stream));
    }
    if (!rc && out->dregion && s->d_region)
        rc = hip_err(launch_region_grad(s->hd.dw, s->d_basew, s->d_region, s->hm.nc,
                                        (int)s->hm.region_scale.size(), out->dregion, s->stream));
    if (!rc && out->dmu && s->hd.n_obst)
        rc = copy_d2d(s, out->dmu, s->hd.dmu, s->hd.n_obst * sizeof(double));
    if (!rc && out->dmu_self) rc = copy_d2d(s, out->dmu_self, s->hd.dmu + kMaxObstacles, sizeof(double));
    if (!rc && out->dforce) {
        if (s->hd.fext) rc = hip_err(launch_permute3(s->hd.dfext, out->dforce, s->d_perm, m, true, s->stream));
        else rc = hip_err(launch_fill(out->dforce, 0.0, 3 * (int64_t)m, s->stream));
    }
    if (!rc && out->dforce_scale && s->T > 0) {
        if (s->hd.fext) rc = copy_d2d(s, out->dforce_scale, s->hd.dfscale, s->T * sizeof(double));
        else rc = hip_err(launch_fill(out->dforce_scale, 0.0, s->T, s->stream));
    }
    return rc;
}

// Warnings of the last backward pass, the most severe first: non-finite state
// gradients, a missed tolerance, a fallback.
int backward_status(sim *s) {
    int rc = mw_check(s);                   // checkpoint segments replayed by the forward kernel
    if (!rc) rc = read_counters(s);
    if (rc) return rc;
    {
        const size_t v3 = 3 * (size_t)s->hd.m;
        std::vector<double> g(2 * v3);
        rc = hip_err(hipMemcpyAsync(g.data(), s->hd.gx, v3 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        if (!rc) rc = hip_err(hipMemcpyAsync(g.data() + v3, s->hd.gv, v3 * sizeof(double), hipMemcpyDeviceToHost,
                                             s->stream));
        if (!rc) rc = hip_err(hipStreamSynchronize(s->stream));
        if (rc) return rc;
        for (double v : g)
            if (!std::isfinite(v)) return SIM_WADJ_NONFINITE;
    }
    if (s->counters_host[3] > 0) return SIM_WADJ_NOCONV;
    if (s->counters_host[2] > 0) return SIM_WADJ_FALLBACK;
    return SIM_OK;
}

}  // namespace

int sim_forward(sim_t *s, int32_t n_steps, double *x_traj_dev, double *xT_dev, double *vT_dev) {
    if (!s || n_steps < 1) return SIM_EINVAL;
    return guarded([&] {
        int rc = prepare_forward(s, n_steps);
        if (!rc) rc = time_mark(s, 0);
        if (!rc) rc = forward_all(s, n_steps, x_traj_dev);
        if (!rc) rc = time_mark(s, 1);
        if (!rc) rc = finish_forward(s, n_steps, xT_dev, vT_dev);
        s->tev_fwd = rc == SIM_OK;
        return rc;
    });
}

int sim_backward(sim_t *s, const double *dL_dxT_dev, const double *dL_dvT_dev, const double *dL_dx_steps_dev,
                 const sim_grads_t *out) {
    if (!s) return SIM_EINVAL;
    if (s->T < 1) return SIM_ESTATE;
    return guarded([&] {
        int rc = prepare_backward(s, dL_dxT_dev, dL_dvT_dev, dL_dx_steps_dev);
        if (!rc) rc = time_mark(s, 2);
        if (!rc) rc = backward_all(s);
        if (!rc) rc = time_mark(s, 3);
        if (!rc) rc = write_grads(s, out);
        if (!rc) rc = backward_status(s);
        s->tev_bwd = rc >= 0;
        return rc;
    });
}

int sim_adjoint_step(sim_t *s, int32_t n, const double *gx_dev, const double *gv_dev, double *dx_dev, double *dv_dev,
                     const sim_grads_t *out) {
    if (!s || !gx_dev || !gv_dev) return SIM_EINVAL;
    if (s->T < 1 || n < 0 || n >= s->T) return SIM_ESTATE;
    if (seg_len(s) > 0) return SIM_ESTATE;      // needs every step's record
    return guarded([&] {
        const int m = s->hd.m;
        int rc = hip_err(launch_permute3(gx_dev, s->hd.gx, s->d_perm, m, false, s->stream));
        if (!rc) rc = hip_err(launch_permute3(gv_dev, s->hd.gv, s->d_perm, m, false, s->stream));
        if (!rc) rc = zero_param_grads(s);
        if (!rc) rc = hip_err(hipMemsetAsync(s->hd.counters, 0, 8 * sizeof(int64_t), s->stream));
        s->hd.gx_steps = nullptr;
        s->hd.step_begin = n;
        s->hd.step_end = n + 1;
        s->hd.rec_step0 = 0;
        if (!rc) rc = factor_steps(s, n, n + 1);
        if (!rc) rc = push_desc(s);
        if (!rc) rc = hip_err(launch_backward(s->dd, 1, s->hd.mixed != 0, s->lds_bwd, bwd_variant(s, s->flags_bwd), 0,
                                              has_mesh(&s, 1), s->stream));
        if (!rc && dx_dev) rc = hip_err(launch_permute3(s->hd.gx, dx_dev, s->d_perm, m, true, s->stream));
        if (!rc && dv_dev) rc = hip_err(launch_permute3(s->hd.gv, dv_dev, s->d_perm, m, true, s->stream));
        if (!rc && out) {
            sim_grads_t o2 = *out;
            o2.dx0 = nullptr;
            o2.dv0 = nullptr;
            rc = write_grads(s, &o2);
        }
        if (!rc) rc = backward_status(s);
        return rc;
    });
}

int sim_state(const sim_t *cs, int32_t n, double *x_dev, double *v_dev) {
    sim *s = const_cast<sim *>(cs);
    if (!s) return SIM_EINVAL;
    if (s->T < 1 || n < 0 || n > s->T) return SIM_ESTATE;
    const int k = seg_len(s);
    return guarded([&] {
        const int m = s->hd.m;
        const size_t v3 = 3 * (size_t)m;
        int rc = SIM_OK;
        int slot = n;
        if (k > 0) {
            const int seg = std::min(n / k, (s->T - 1) / k), a = seg * k, b = std::min(s->T, a + k);
            rc = load_ckpt(s, seg);
            if (!rc) rc = run_forward_range(s, a, b);
            if (!rc) rc = mw_check(s);
            slot = n - a;
        }
        if (!rc && x_dev) rc = hip_err(launch_permute3(s->hd.rec_x + slot * v3, x_dev, s->d_perm, m, true, s->stream));
        if (!rc && v_dev) rc = hip_err(launch_permute3(s->hd.rec_v + slot * v3, v_dev, s->d_perm, m, true, s->stream));
        if (!rc) rc = hip_err(hipStreamSynchronize(s->stream));
        return rc;
    });
}

int sim_modes(const sim_t *cs, int32_t n, uint8_t *modes_host) {
    sim *s = const_cast<sim *>(cs);
    if (!s || !modes_host) return SIM_EINVAL;
    if (s->T < 1 || n < 0 || n >= s->T) return SIM_ESTATE;
    const int k = seg_len(s);
    return guarded([&] {
        const int m = s->hd.m;
        int rc = SIM_OK;
        int slot = n;
        if (k > 0) {                        // recompute the segment holding step n
            const int seg = n / k, a = seg * k, b = std::min(s->T, a + k);
            rc = load_ckpt(s, seg);
            if (!rc) rc = run_forward_range(s, a, b);
            if (!rc) rc = mw_check(s);
            slot = n - a;
        }
        if (!rc) rc = hip_err(launch_modes(s->hd.rec_mode + (size_t)slot * m, s->d_modes_tmp, s->d_perm, m, s->stream));
        if (!rc) rc = hip_err(hipMemcpyAsync(modes_host, s->d_modes_tmp, m, hipMemcpyDeviceToHost, s->stream));
        if (!rc) rc = hip_err(hipStreamSynchronize(s->stream));
        return rc;
    });
}

int sim_self_pairs(const sim_t *cs, int32_t n, int32_t *partner_host) {
    sim *s = const_cast<sim *>(cs);
    if (!s || !partner_host) return SIM_EINVAL;
    if (s->T < 1) return SIM_ESTATE;
    if (n < 0 || n >= s->T) return SIM_EINVAL;
    const int k = seg_len(s);
    return guarded([&] {
        const int m = s->hd.m;
        if (!s->hd.self_on) {
            std::fill(partner_host, partner_host + m, -1);
            return SIM_OK;
        }
        int rc = SIM_OK;
        int slot = n;
        if (k > 0) {                        // recompute the segment holding step n
            const int seg = n / k, a = seg * k, b = std::min(s->T, a + k);
            rc = load_ckpt(s, seg);
            if (!rc) rc = run_forward_range(s, a, b);
            if (!rc) rc = mw_check(s);
            slot = n - a;
        }
        std::vector<int32_t> p(m);
        if (!rc)
            rc = hip_err(hipMemcpyAsync(p.data(), s->hd.rec_partner + (size_t)slot * m, m * sizeof(int32_t),
                                        hipMemcpyDeviceToHost, s->stream));
        if (!rc) rc = hip_err(hipStreamSynchronize(s->stream));
        if (!rc)
            for (int i = 0; i < m; ++i) partner_host[s->hm.perm[i]] = p[i] >= 0 ? s->hm.perm[p[i]] : -1;
        return rc;
    });
}

int sim_stats(const sim_t *cs, sim_stats_t *out) {
    if (!cs || !out) return SIM_EINVAL;
    const sim *s = cs;
    std::memset(out, 0, sizeof(*out));
    out->n_nodes = s->hm.m;
    out->n_edges = s->hm.n_edges;
    out->n_bend = s->hm.n_bend;
    out->n_constraints_active = s->nca;
    out->nnz_P = (int64_t)s->hm.ks_col.size();
    out->nnz_L = s->hm.nnz_L;
    out->n_supernodes = s->hm.ns;
    out->n_levels = s->hm.n_levels;
    out->steps_recorded = s->T;
    out->fwd_iters_total = s->counters_host[0];
    out->adj_iters_total = s->counters_host[1];
    out->adj_fallbacks = (int32_t)s->counters_host[2];
    out->adj_noconv = (int32_t)s->counters_host[3];
    out->device_bytes = s->bytes;
    out->adj_krylov_total = s->counters_host[4];
    out->factor_bytes = s->factor_bytes;
    out->lds_forward = (int64_t)s->lds_fwd;
    out->lds_backward = (int64_t)s->lds_bwd;
    out->adj_factor_bytes = s->hd.af_size * (int64_t)sizeof(double);
    out->adj_pivot_perturbed = s->counters_host[5];
    out->fwd_launches = s->fwd_launches;
    out->lds_flags_fwd = s->flags_fwd;
    out->fwd_workgroups = s->hd.mw >= 2 ? s->hd.mw : 1;
    out->lds_flags_bwd = s->flags_bwd;
    if (s->tev_fwd) {
        float ms = 0.0f;
        if (hipEventSynchronize(s->tev[1]) == hipSuccess && hipEventElapsedTime(&ms, s->tev[0], s->tev[1]) == hipSuccess)
            out->fwd_ms = ms;
    }
    if (s->tev_bwd) {
        float ms = 0.0f;
        if (hipEventSynchronize(s->tev[3]) == hipSuccess && hipEventElapsedTime(&ms, s->tev[2], s->tev[3]) == hipSuccess)
            out->bwd_ms = ms;
    }
    if (s->T > 0 && s->hd.step_info) {
        return guarded([&] {
            std::vector<int32_t> info(4 * (size_t)s->T);
            int rc = hip_err(hipMemcpyAsync(info.data(), s->hd.step_info, info.size() * sizeof(int32_t),
                                            hipMemcpyDeviceToHost, s->stream));
            if (!rc) rc = hip_err(hipStreamSynchronize(s->stream));
            if (rc) return rc;
            int64_t contact = 0;
            for (int n = 0; n < s->T; ++n) {
                out->fwd_iters_max = std::max(out->fwd_iters_max, info[4 * n]);
                for (int q = 1; q < 4; ++q) {
                    out->mode_counts[q] += info[4 * n + q];
                    contact += info[4 * n + q];
                }
            }
            out->mode_counts[SIM_MODE_FREE] = (int64_t)s->T * s->hm.m - contact;
            return SIM_OK;
        });
    }
    return SIM_OK;
}

int sim_step_stats(const sim_t *cs, int32_t n, int32_t *out) {
    if (!cs || !out) return SIM_EINVAL;
    const sim *s = cs;
    if (s->T < 1 || !s->hd.step_info) return SIM_ESTATE;
    if (n < 0 || n >= s->T) return SIM_EINVAL;
    int rc = hip_err(hipMemcpyAsync(out, s->hd.step_info + 4 * (size_t)n, 4 * sizeof(int32_t), hipMemcpyDeviceToHost,
                                    s->stream));
    if (!rc) rc = hip_err(hipStreamSynchronize(s->stream));
    return rc;
}

// Scratch layout of the allocation-free forward (byte offsets, 256-aligned).
struct NoallocLayout {
    size_t desc, ctr, red, x, v, vk, vk1, rhs, b0, f, ubar, cfr, wp, ubuf, rx, rv, rub, mode, cobst, rmode, robst;
    size_t ybuf, cand, partner, rpartner, shead, snext;   // node-node contact (self-collision on)
    size_t total;
};

NoallocLayout noalloc_layout(const sim *s) {
    const size_t m = (size_t)s->hd.m, d = sizeof(double);
    NoallocLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += (std::max<size_t>(bytes, 8) + 255) & ~size_t(255);
        return at;
    };
    L.desc = take(sizeof(SimDev));
    L.ctr = take(16 * sizeof(int64_t));          // counters [0, 8), forward position at 8
    L.red = take(64 * d);
    L.x = take(3 * m * d);
    L.v = take(3 * m * d);
    L.vk = take(3 * m * d);
    L.vk1 = take(3 * m * d);
    L.rhs = take(3 * m * d);
    L.b0 = take(3 * m * d);
    L.f = take(3 * m * d);
    L.ubar = take(3 * m * d);
    L.cfr = take(8 * m * d);
    L.wp = take(3 * (size_t)std::max(s->nca, 1) * d);
    L.ubuf = take((size_t)std::max(s->hd.n_ubuf, 1) * d);
    L.rx = take(2 * 3 * m * d);
    L.rv = take(2 * 3 * m * d);
    L.rub = take(3 * m * d);
    L.mode = take(m);
    L.cobst = take(m);
    L.rmode = take(m);
    L.robst = take(m);
    if (s->hd.self_on) {
        L.ybuf = take(3 * m * d);
        L.cand = take(m * sizeof(int32_t));
        L.partner = take(m * sizeof(int32_t));
        L.rpartner = take(m * sizeof(int32_t));
        L.shead = take((size_t)(s->hd.self_hmask + 1) * sizeof(int32_t));
        L.snext = take(m * sizeof(int32_t));
    }
    L.total = o;
    return L;
}

int sim_forward_noalloc(sim_t *s, int32_t n_steps, double *xT_dev, double *vT_dev) {
    if (!s || n_steps < 1 || !xT_dev || !vT_dev) return SIM_EINVAL;
    if (s->hd.fscale && n_steps > s->n_fscale) return SIM_EINVAL;    // multipliers run out
    const NoallocLayout L = noalloc_layout(s);
    if (L.total > kNoallocScratchBytes) return SIM_ESCRATCH;
    void *base = nullptr;
    int rc = hip_err(noalloc_scratch(&base));
    if (rc) return rc;
    char *b = (char *)base;
    const int m = s->hd.m;
    const size_t v3b = 3 * (size_t)m * sizeof(double);
    SimDev &d = s->hd_noalloc;
    d = s->hd;                                   // the handle's tables; its work memory replaced below
    d.counters = (int64_t *)(b + L.ctr);
    d.fwd_pos = (int64_t *)(b + L.ctr) + 8;
    d.red = (double *)(b + L.red);
    d.x = (double *)(b + L.x);
    d.v = (double *)(b + L.v);
    d.vk = (double *)(b + L.vk);
    d.vk1 = (double *)(b + L.vk1);
    d.rhs = (double *)(b + L.rhs);
    d.b0 = (double *)(b + L.b0);
    d.f = (double *)(b + L.f);
    d.ubar = (double *)(b + L.ubar);
    d.cfr = (double *)(b + L.cfr);
    d.wp = (double *)(b + L.wp);
    d.ubuf = (double *)(b + L.ubuf);
    d.rec_x = (double *)(b + L.rx);
    d.rec_v = (double *)(b + L.rv);
    d.rec_ubar = (double *)(b + L.rub);
    d.mode = (uint8_t *)(b + L.mode);
    d.cobst = (int8_t *)(b + L.cobst);
    d.rec_mode = (uint8_t *)(b + L.rmode);
    d.rec_obst = (int8_t *)(b + L.robst);
    if (d.self_on) {
        d.ybuf = (double *)(b + L.ybuf);
        d.cand = (int32_t *)(b + L.cand);
        d.partner = (int32_t *)(b + L.partner);
        d.rec_partner = (int32_t *)(b + L.rpartner);
        d.self_head = (int32_t *)(b + L.shead);
        d.self_next = (int32_t *)(b + L.snext);
    }
    d.rec_cap = 1;
    d.rec_ring = 1;
    d.step_info = nullptr;
    d.step_begin = 0;
    d.step_end = n_steps;
    d.rec_step0 = 0;
    d.fwd_epoch = 0;
    SimDev *dd = (SimDev *)(b + L.desc);
    // everything below is enqueued on the handle's stream; nothing allocates,
    // synchronises or clears memory with a memset (the call may be captured)
    rc = hip_err(hipMemcpyAsync(dd, &d, sizeof(SimDev), hipMemcpyHostToDevice, s->stream));
    if (!rc) rc = hip_err(launch_fill((double *)(b + L.ctr), 0.0, 16, s->stream));
    if (!rc) rc = hip_err(launch_fill(d.ubar, 0.0, 3 * (int64_t)m, s->stream));
    if (!rc) rc = hip_err(launch_fill(d.f, 0.0, 3 * (int64_t)m, s->stream));        // warm start of step 0
    if (!rc) rc = copy_d2d(s, d.x, s->start_x, v3b);
    if (!rc) rc = copy_d2d(s, d.v, s->start_v, v3b);
    if (!rc) rc = hip_err(launch_forward(dd, 1, s->hd.mixed != 0, s->lds_fwd, s->flags_fwd, 0, has_mesh(&s, 1),
                                         s->stream));
    if (!rc) rc = hip_err(launch_permute3(d.x, xT_dev, s->d_perm, m, true, s->stream));
    if (!rc) rc = hip_err(launch_permute3(d.v, vT_dev, s->d_perm, m, true, s->stream));
    return rc;
}

int64_t sim_noalloc_scratch_bytes(const sim_t *s) {
    return s ? (int64_t)noalloc_layout(s).total : -1;
}

int sim_batch_forward(sim_t *const *sims, int32_t n, const int32_t *n_steps, double *const *xT_dev,
                      double *const *vT_dev) {
    if (!sims || n < 1 || !n_steps) return SIM_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!sims[i] || n_steps[i] < 1) return SIM_EINVAL;
        if (seg_len(sims[i]) > 0) return SIM_EINVAL;   // batched passes keep every record
        if (sims[i]->stream != sims[0]->stream || sims[i]->hd.mixed != sims[0]->hd.mixed) return SIM_EINVAL;
    }
    sim *s0 = sims[0];
    return guarded([&] {
        std::vector<SimDev> descs(n);
        int rc = SIM_OK;
        for (int i = 0; i < n && !rc; ++i) {
            rc = prepare_forward(sims[i], n_steps[i]);
            sims[i]->hd.step_begin = 0;
            sims[i]->hd.step_end = n_steps[i];
            sims[i]->hd.rec_step0 = 0;
            ++sims[i]->hd.fwd_epoch;
            descs[i] = sims[i]->hd;
            if (!rc) rc = push_desc(sims[i]);
        }
        if (rc) return rc;
        SimDev *d = batch_descs(s0, n);
        rc = hip_err(hipMemcpyAsync(d, descs.data(), n * sizeof(SimDev), hipMemcpyHostToDevice, s0->stream));
        int fl = 0;
        const size_t lb = batch_lds(sims, n, true, fl);
        if (!rc) rc = hip_err(launch_forward(d, n, s0->hd.mixed != 0, lb, fl, fwd_helpers(sims, n), has_mesh(sims, n),
                                             s0->stream));
        for (int i = 0; i < n && !rc; ++i)
            rc = finish_forward(sims[i], n_steps[i], xT_dev ? xT_dev[i] : nullptr, vT_dev ? vT_dev[i] : nullptr);
        (void)hipStreamSynchronize(s0->stream);
        return rc;
    });
}

int sim_batch_backward(sim_t *const *sims, int32_t n, const double *const *dL_dxT_dev, const sim_grads_t *out) {
    if (!sims || n < 1) return SIM_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!sims[i]) return SIM_EINVAL;
        if (sims[i]->T < 1) return SIM_ESTATE;
        if (seg_len(sims[i]) > 0 || sims[i]->stream != sims[0]->stream || sims[i]->hd.mixed != sims[0]->hd.mixed ||
            sims[i]->hd.adj_direct != sims[0]->hd.adj_direct)
            return SIM_EINVAL;
    }
    sim *s0 = sims[0];
    return guarded([&] {
        std::vector<SimDev> descs(n);
        std::vector<int32_t> work;           // (handle, slot) of every step factor (direct adjoint)
        int rc = SIM_OK;
        for (int i = 0; i < n && !rc; ++i) {
            rc = fac_idle(sims[i]);                 // its step factors are redone below
            if (!rc) rc = prepare_backward(sims[i], dL_dxT_dev ? dL_dxT_dev[i] : nullptr, nullptr, nullptr);
            sims[i]->hd.step_begin = 0;
            sims[i]->hd.step_end = sims[i]->T;
            sims[i]->hd.rec_step0 = 0;
            if (sims[i]->hd.adj_direct) {
                ensure_af(sims[i], sims[i]->T);
                sims[i]->hd.af_step0 = 0;
                for (int k = 0; k < sims[i]->T; ++k) { work.push_back(i); work.push_back(k); }
            }
            descs[i] = sims[i]->hd;
            if (!rc) rc = push_desc(sims[i]);
        }
        if (rc) return rc;
        SimDev *d = batch_descs(s0, n);
        rc = hip_err(hipMemcpyAsync(d, descs.data(), n * sizeof(SimDev), hipMemcpyHostToDevice, s0->stream));
        if (!rc && !work.empty()) rc = factor_pairs(s0, d, std::vector<sim *>(sims, sims + n), work, s0->stream);
        int fl = 0;
        const size_t lb = batch_lds(sims, n, false, fl);
        if (!rc) rc = hip_err(launch_backward(d, n, s0->hd.mixed != 0, lb, bwd_variant(s0, fl), 0, has_mesh(sims, n),
                                              s0->stream));
        int warn = SIM_OK;
        for (int i = 0; i < n && !rc; ++i) {
            if (out) rc = write_grads(sims[i], &out[i]);
            if (!rc) {
                int st = backward_status(sims[i]);
                if (st < 0) rc = st;
                else if (st > warn) warn = st;
            }
        }
        (void)hipStreamSynchronize(s0->stream);
        return rc ? rc : warn;
    });
}



int sim_trim(sim_t *s) {
    if (!s) return SIM_EINVAL;
    int rc = hip_err(hipStreamSynchronize(s->stream));
    if (!rc) rc = fac_idle(s);
    if (rc) return rc;
    for (void **p : {(void **)&s->hd.rec_x, (void **)&s->hd.rec_v, (void **)&s->hd.rec_ubar, (void **)&s->hd.rec_mode,
                     (void **)&s->hd.rec_obst, (void **)&s->ckpt, (void **)&s->gsteps, (void **)&s->hd.af,
                     (void **)&s->hd.af_ws, (void **)&s->d_work, (void **)&s->batch_desc,
                     (void **)&s->hd.step_info}) {
        dev_release(s, *p);
        *p = nullptr;
    }
    s->batch_desc_cap = 0;
    s->step_info_cap = 0;
    s->hd.rec_cap = 0;
    s->ckpt_cap = 0;
    s->gsteps_cap = 0;
    s->af_cap = 0;
    s->work_cap = 0;
    s->T = -1;
    s->phase = 0;
    return SIM_OK;
}

int sim_job_forward(sim_t *s, int32_t n_steps) {
    if (!s || n_steps < 1) return SIM_EINVAL;
    if (seg_len(s) > 0) return SIM_EINVAL;
    return guarded([&] {
        int rc = prepare_forward(s, n_steps);
        if (rc) return rc;
        s->T = -1;
        s->phase = 1;
        s->cursor = 0;
        s->target = n_steps;
        return SIM_OK;
    });
}

int sim_job_backward(sim_t *s, const double *dL_dxT_dev, const double *dL_dvT_dev) {
    if (!s) return SIM_EINVAL;
    if (s->phase != 2 || s->T < 1) return SIM_ESTATE;
    return guarded([&] {
        int rc = fac_idle(s);                       // the job refactors its steps chunk by chunk
        if (!rc) rc = prepare_backward(s, dL_dxT_dev, dL_dvT_dev, nullptr);
        if (rc) return rc;
        s->phase = 3;
        s->cursor = s->T;
        return SIM_OK;
    });
}

int sim_batch_advance(sim_t *const *sims, int32_t n, const int32_t *steps, void *backward_stream, int32_t *left) {
    if (!sims || n < 1 || !steps) return SIM_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!sims[i] || steps[i] < 1) return SIM_EINVAL;
        if (sims[i]->stream != sims[0]->stream || sims[i]->hd.mixed != sims[0]->hd.mixed ||
            sims[i]->hd.adj_direct != sims[0]->hd.adj_direct)
            return SIM_EINVAL;
        if (sims[i]->phase != 1 && sims[i]->phase != 3) return SIM_ESTATE;
    }
    hipStream_t sf = sims[0]->stream, sb = backward_stream ? (hipStream_t)backward_stream : sf;
    return guarded([&] {
        std::vector<sim *> fw, bw;
        std::vector<SimDev> df, db;
        std::vector<int32_t> pairs;
        int rc = SIM_OK;
        for (int i = 0; i < n; ++i) {
            sim *h = sims[i];
            if (h->phase == 1) {
                h->hd.step_begin = h->cursor;
                h->hd.step_end = std::min(h->target, h->cursor + steps[i]);
                h->hd.rec_step0 = 0;
                ++h->hd.fwd_epoch;
                fw.push_back(h);
                df.push_back(h->hd);
            } else {
                const int lo = std::max(0, h->cursor - steps[i]);
                h->hd.step_begin = lo;
                h->hd.step_end = h->cursor;
                h->hd.rec_step0 = 0;
                if (h->hd.adj_direct) {
                    ensure_af(h, h->cursor - lo);
                    h->hd.af_step0 = lo;
                    for (int k = 0; k < h->cursor - lo; ++k) {
                        pairs.push_back((int32_t)bw.size());
                        pairs.push_back(k);
                    }
                }
                bw.push_back(h);
                db.push_back(h->hd);
            }
        }
        SimDev *room = batch_descs(sims[0], fw.size() + bw.size());
        SimDev *dfd = fw.empty() ? nullptr : room;
        SimDev *dbd = bw.empty() ? nullptr : room + fw.size();
        if (dfd) rc = hip_err(hipMemcpyAsync(dfd, df.data(), df.size() * sizeof(SimDev), hipMemcpyHostToDevice, sf));
        if (!rc && dbd) rc = hip_err(hipMemcpyAsync(dbd, db.data(), db.size() * sizeof(SimDev), hipMemcpyHostToDevice, sf));
        if (!rc) rc = hip_err(hipStreamSynchronize(sf));          // descriptors in place before either stream uses them
        if (!rc && dfd) {
            int fl = 0;
            const size_t lb = batch_lds(fw.data(), (int)fw.size(), true, fl);
            rc = hip_err(launch_forward(dfd, (int)fw.size(), fw[0]->hd.mixed != 0, lb, fl, fwd_helpers(fw.data(), (int)fw.size()),
                                        has_mesh(fw.data(), (int)fw.size()),
                                        sf));
        }
        if (!rc && dbd) {
            if (!pairs.empty()) rc = factor_pairs(bw[0], dbd, bw, pairs, sb);
            int fl = 0;
            const size_t lb = batch_lds(bw.data(), (int)bw.size(), false, fl);
            if (!rc) rc = hip_err(launch_backward(dbd, (int)bw.size(), bw[0]->hd.mixed != 0, lb, bwd_variant(bw[0], fl), 0,
                                                  has_mesh(bw.data(), (int)bw.size()), sb));
        }
        const int r1 = hip_err(hipStreamSynchronize(sf));
        const int r2 = hip_err(hipStreamSynchronize(sb));
        if (!rc) rc = r1 ? r1 : r2;
        if (rc) return rc;
        for (sim *h : fw) {
            h->cursor = h->hd.step_end;
            if (h->cursor == h->target) {
                rc = read_counters(h);
                if (rc) return rc;
                h->T = h->target;
                h->phase = 2;
            }
        }
        for (sim *h : bw) {
            h->cursor = h->hd.step_begin;
            if (h->cursor == 0) h->phase = 4;
        }
        if (left)
            for (int i = 0; i < n; ++i)
                left[i] = sims[i]->phase == 1 ? sims[i]->target - sims[i]->cursor
                                              : sims[i]->phase == 3 ? sims[i]->cursor : 0;
        return SIM_OK;
    });
}

int sim_job_grads(sim_t *s, const sim_grads_t *out) {
    if (!s) return SIM_EINVAL;
    if (s->phase != 4) return SIM_ESTATE;
    return guarded([&] {
        int rc = write_grads(s, out);
        if (!rc) rc = backward_status(s);
        if (rc >= 0) s->phase = 2;                  // the recorded forward stays valid
        return rc;
    });
}

void sim_destroy(sim_t *s) {
    if (!s) return;
    if (s->stream || !s->owned.empty()) (void)hipStreamSynchronize(s->stream);
    if (s->fac_stream) {
        (void)hipStreamSynchronize(s->fac_stream);
        (void)hipEventDestroy(s->fac_ev);
        (void)hipEventDestroy(s->fac_done);
        (void)hipStreamDestroy(s->fac_stream);
    }
    for (auto [p, nb] : s->owned) {
        if (s->free_fn) s->free_fn(p, s->ctx);
        else (void)hipFree(p);
    }
    s->owned.clear();
    for (hipEvent_t &e : s->tev)
        if (e) (void)hipEventDestroy(e);
    delete s;
}

const char *sim_strerror(int code) {
    switch (code) {
        case SIM_OK: return "ok";
        case SIM_EINVAL: return "invalid mesh or parameters";
        case SIM_ESYNC: return "a multi-workgroup forward launch gave up waiting at a barrier";
        case SIM_ESCRATCH: return "the mesh needs more than the 16 MiB of device scratch of sim_forward_noalloc";
        case SIM_ENOTSPD: return "PD matrix is not positive definite";
        case SIM_ENOMEM: return "out of memory";
        case SIM_ENONFINITE: return "non-finite input or state";
        case SIM_ESTATE: return "call out of order (no recorded rollout or bad step)";
        case SIM_EHIP: return "HIP runtime error";
        case SIM_WADJ_FALLBACK: return "warning: an adjoint step used the fallback solver";
        case SIM_WADJ_NOCONV: return "warning: an adjoint step missed its tolerance";
        case SIM_WADJ_NONFINITE: return "warning: the state gradients overflowed (not finite)";
        default: return "unknown code";
    }
}

int sim_analyze(const sim_mesh_t *mesh, const sim_params_t *params, int32_t leaf_size, sim_stats_t *stats,
                int32_t *perm_out, double *dense_L_out, int32_t max_dense) {
    return guarded([&]() -> int {
    HostModel hm;
    int rc = hm.build(mesh, params);
    if (rc) return rc;
    rc = hm.order_and_factor(leaf_size > 0 ? leaf_size : 32, merge_cap_default());
    if (rc) return rc;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->n_nodes = hm.m;
        stats->n_edges = hm.n_edges;
        stats->n_bend = hm.n_bend;
        int nca = 0;
        for (double r : hm.rho) nca += r > 0;
        stats->n_constraints_active = nca;
        stats->nnz_P = (int64_t)hm.ks_col.size();
        stats->nnz_L = hm.nnz_L;
        stats->n_supernodes = hm.ns;
        stats->n_levels = hm.n_levels;
        stats->steps_recorded = -1;
    }
    if (perm_out) std::memcpy(perm_out, hm.perm.data(), hm.m * sizeof(int32_t));
    if (dense_L_out && hm.m <= max_dense) hm.dense_L(dense_L_out);
    return SIM_OK;
    });
}

}  // extern "C"
