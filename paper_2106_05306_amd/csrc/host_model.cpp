// Host setup of one cloth: constraint tables (springs, cotangent bending,
// attachments), the scalar PD matrix P_s (P = P_s (x) I_3), a nested-dissection
// ordering, and a supernodal float64 Cholesky factor of P_s.
#include "host_model.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <utility>

namespace dc {

namespace {

inline void sub3(const double *a, const double *b, double *o) {
    o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline double norm3(const double *a) { return std::sqrt(dot3(a, a)); }

bool finite_all(const double *p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace

int HostModel::build(const sim_mesh_t *mesh, const sim_params_t *p) {
    if (!mesh || !p || mesh->n_nodes < 1 || !mesh->X || mesh->n_tris < 1 || !mesh->tris) {
        error = "mesh needs nodes and triangles";
        return SIM_EINVAL;
    }
    m = mesh->n_nodes;
    X.assign(mesh->X, mesh->X + 3 * (size_t)m);
    if (!finite_all(X.data(), X.size())) { error = "non-finite rest positions"; return SIM_ENONFINITE; }
    if (!p->node_mass) { error = "node_mass is required"; return SIM_EINVAL; }
    mass.assign(p->node_mass, p->node_mass + m);
    for (double v : mass)
        if (!(v > 0) || !std::isfinite(v)) { error = "masses must be positive and finite"; return SIM_ENOTSPD; }
    if (!(p->h > 0) || !std::isfinite(p->h)) { error = "time step must be positive"; return SIM_EINVAL; }
    h = p->h;
    for (int d = 0; d < 3; ++d) g[d] = p->gravity[d];
    pd_iters = p->pd_iters;
    fwd_tol = p->fwd_tol;
    warm_start = p->warm_start ? 1 : 0;
    fwd_max_iters = p->fwd_max_iters > 0 ? p->fwd_max_iters : 100000;
    if (fwd_tol <= 0 && pd_iters < 1) { error = "pd_iters must be >= 1"; return SIM_EINVAL; }
    adj_tol = p->adj_tol > 0 ? p->adj_tol : 1e-10;
    adj_max_iters = p->adj_max_iters > 0 ? p->adj_max_iters : 500;
    precision = p->precision;
    if (precision != SIM_FP64 && precision != SIM_MIXED) { error = "bad precision"; return SIM_EINVAL; }
    checkpoint_every = std::max(0, p->checkpoint_every);
    adj_restart = p->adj_restart > 0 ? std::min(p->adj_restart, 60) : 60;
    adj_solver = p->adj_solver;
    adj_window = std::max(0, p->adj_window);
    if (adj_solver != SIM_ADJ_ITERATIVE && adj_solver != SIM_ADJ_DIRECT) { error = "bad adj_solver"; return SIM_EINVAL; }
    self_d = p->self_thickness;
    self_r = p->self_radius > 0 ? p->self_radius : p->self_thickness;
    self_mu = p->self_mu;
    if (!(self_d >= 0) || !std::isfinite(self_d) || !(p->self_radius >= 0) || !std::isfinite(p->self_radius) ||
        !(self_mu >= 0) || !std::isfinite(self_mu)) {
        error = "self-collision thickness, radius and friction must be finite and >= 0";
        return SIM_EINVAL;
    }
    if (self_d > 0 && adj_solver == SIM_ADJ_DIRECT) {
        error = "self-collision needs the iterative adjoint (pair blocks lie outside the factor's pattern)";
        return SIM_EINVAL;
    }
    if (p->n_obstacles < 0 || p->n_obstacles > 8 || (p->n_obstacles > 0 && !p->obstacles)) {
        error = "0..8 obstacles";
        return SIM_EINVAL;
    }
    obstacles.assign(p->obstacles, p->obstacles + p->n_obstacles);
    for (auto &o : obstacles) {
        if (o.type == SIM_PLANE) {
            double nn = norm3(o.n);
            if (!(nn > 0)) { error = "plane normal is zero"; return SIM_EINVAL; }
            for (int d = 0; d < 3; ++d) o.n[d] /= nn;
        } else if (o.type == SIM_SPHERE) {
            if (!(o.radius > 0)) { error = "sphere radius must be positive"; return SIM_EINVAL; }
        } else if (o.type == SIM_MESH) {
            if (o.n_verts < 3 || o.n_tris < 1 || o.n_tris > 65536 || !o.verts || !o.tris) {
                error = "mesh obstacle needs vertices and 1..65536 triangles";
                return SIM_EINVAL;
            }
        } else {
            error = "unknown obstacle type";
            return SIM_EINVAL;
        }
        if (!(o.mu >= 0) || !std::isfinite(o.mu)) { error = "friction must be >= 0"; return SIM_EINVAL; }
    }
    obst_tri.assign(obstacles.size(), {});
    obst_closed.assign(obstacles.size(), 0);
    obst_ball.assign(4 * obstacles.size(), 0.0);
    for (size_t k = 0; k < obstacles.size(); ++k) {
        sim_obstacle_t &o = obstacles[k];
        if (o.type == SIM_MESH) {
            std::vector<double> &tri = obst_tri[k];
            tri.resize(16 * (size_t)o.n_tris);
            for (int t = 0; t < o.n_tris; ++t) {
                const double *v[3];
                for (int r = 0; r < 3; ++r) {
                    const int32_t vi = o.tris[3 * t + r];
                    if (vi < 0 || vi >= o.n_verts) { error = "mesh obstacle: vertex index out of range"; return SIM_EINVAL; }
                    v[r] = o.verts + 3 * (size_t)vi;
                    for (int d = 0; d < 3; ++d) {
                        if (!std::isfinite(v[r][d])) { error = "mesh obstacle: non-finite vertex"; return SIM_EINVAL; }
                        tri[16 * t + 3 * r + d] = v[r][d];
                    }
                }
                const double u[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
                const double w[3] = {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
                double nn[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
                const double ln = norm3(nn);
                if (!(ln > 0)) { error = "mesh obstacle: degenerate triangle"; return SIM_EINVAL; }
                for (int d = 0; d < 3; ++d) tri[16 * t + 9 + d] = nn[d] / ln;
                // bounding ball: the centroid and the largest vertex distance (+ margin)
                double c[3], rb = 0.0;
                for (int d = 0; d < 3; ++d) c[d] = (v[0][d] + v[1][d] + v[2][d]) / 3.0;
                for (int r = 0; r < 3; ++r) {
                    const double e[3] = {v[r][0] - c[0], v[r][1] - c[1], v[r][2] - c[2]};
                    rb = std::max(rb, norm3(e));
                }
                for (int d = 0; d < 3; ++d) tri[16 * t + 12 + d] = c[d];
                tri[16 * t + 15] = rb * (1.0 + 1e-12) + 1e-300;
            }
        }
        if (o.type == SIM_MESH) {
            // closed: each directed edge appears once and its reverse once
            std::map<std::pair<int, int>, int> de;
            for (int t = 0; t < o.n_tris; ++t)
                for (int r = 0; r < 3; ++r) ++de[{o.tris[3 * t + r], o.tris[3 * t + (r + 1) % 3]}];
            bool closed = true;
            for (const auto &kv : de) {
                auto it = de.find({kv.first.second, kv.first.first});
                if (kv.second != 1 || it == de.end() || it->second != 1) { closed = false; break; }
            }
            double c[3] = {0, 0, 0}, r = 0;
            for (int v = 0; v < o.n_verts; ++v)
                for (int d = 0; d < 3; ++d) c[d] += o.verts[3 * v + d] / o.n_verts;
            for (int v = 0; v < o.n_verts; ++v) {
                const double e[3] = {o.verts[3 * v] - c[0], o.verts[3 * v + 1] - c[1], o.verts[3 * v + 2] - c[2]};
                r = std::max(r, norm3(e));
            }
            obst_closed[k] = closed ? 1 : 0;
            for (int d = 0; d < 3; ++d) obst_ball[4 * k + d] = c[d];
            obst_ball[4 * k + 3] = r * (1.0 + 1e-12) + 1e-12;    // rounding margin
        }
        o.verts = nullptr;                    // the caller's arrays are not kept
        o.tris = nullptr;
    }

    // ---------------------------------------------------------------- triangles
    const int nt = mesh->n_tris;
    for (int t = 0; t < 3 * nt; ++t)
        if (mesh->tris[t] < 0 || mesh->tris[t] >= m) { error = "triangle index out of range"; return SIM_EINVAL; }
    // edge -> (count, cotangent weight sum); keyed by (min, max)
    std::map<std::pair<int, int>, std::pair<int, double>> ew;
    for (int t = 0; t < nt; ++t) {
        const int32_t *tri = mesh->tris + 3 * t;
        for (int r = 0; r < 3; ++r) {
            int i = tri[r], j = tri[(r + 1) % 3], k = tri[(r + 2) % 3];
            double u[3], v[3], c[3];
            sub3(&X[3 * i], &X[3 * k], u);
            sub3(&X[3 * j], &X[3 * k], v);
            c[0] = u[1] * v[2] - u[2] * v[1];
            c[1] = u[2] * v[0] - u[0] * v[2];
            c[2] = u[0] * v[1] - u[1] * v[0];
            double cn = norm3(c);
            if (!(cn > 0)) { error = "degenerate triangle"; return SIM_EINVAL; }
            auto key = std::make_pair(std::min(i, j), std::max(i, j));
            auto &e = ew[key];
            e.first += 1;
            e.second += 0.5 * dot3(u, v) / cn;       // half the cotangent of the angle at k
        }
    }
    // springs
    if (mesh->n_edges > 0) {
        if (!mesh->edges) { error = "n_edges > 0 needs an edge list"; return SIM_EINVAL; }
        n_edges = mesh->n_edges;
        edges.assign(mesh->edges, mesh->edges + 2 * (size_t)n_edges);
        for (int e = 0; e < n_edges; ++e) {
            int a = edges[2 * e], b = edges[2 * e + 1];
            if (a < 0 || b < 0 || a >= m || b >= m || a == b) { error = "bad edge"; return SIM_EINVAL; }
        }
    } else {
        n_edges = (int)ew.size();
        edges.resize(2 * (size_t)n_edges);
        int e = 0;
        for (auto &kv : ew) { edges[2 * e] = kv.first.first; edges[2 * e + 1] = kv.first.second; ++e; }
    }
    if (!p->edge_stiffness) { error = "edge_stiffness is required"; return SIM_EINVAL; }
    // bending: interior vertices (every incident edge shared by two triangles)
    std::vector<char> boundary(m, 0), touched(m, 0);
    for (auto &kv : ew) {
        touched[kv.first.first] = touched[kv.first.second] = 1;
        if (kv.second.first == 1) boundary[kv.first.first] = boundary[kv.first.second] = 1;
    }
    std::vector<std::vector<std::pair<int, double>>> nbr(m);
    for (auto &kv : ew) {
        int a = kv.first.first, b = kv.first.second;
        nbr[a].push_back({b, kv.second.second});
        nbr[b].push_back({a, kv.second.second});
    }
    bend_center.clear();
    for (int j = 0; j < m; ++j)
        if (touched[j] && !boundary[j]) bend_center.push_back(j);
    n_bend = (int)bend_center.size();
    nc = n_edges + n_bend;

    // stencils (caller ids)
    c_ptr.assign(1, 0);
    c_node.clear();
    c_coef.clear();
    for (int e = 0; e < n_edges; ++e) {
        c_node.push_back(edges[2 * e]);     c_coef.push_back(1.0);
        c_node.push_back(edges[2 * e + 1]); c_coef.push_back(-1.0);
        c_ptr.push_back((int32_t)c_node.size());
    }
    for (int b = 0; b < n_bend; ++b) {
        int j = bend_center[b];
        auto nb = nbr[j];
        std::sort(nb.begin(), nb.end());
        double tot = 0;
        for (auto &pr : nb) {
            if (pr.second == 0.0) continue;          // e.g. right angles opposite grid diagonals
            c_node.push_back(pr.first);
            c_coef.push_back(pr.second);
            tot += pr.second;
        }
        c_node.push_back(j);
        c_coef.push_back(-tot);
        c_ptr.push_back((int32_t)c_node.size());
    }
    // weights, regions
    base_w.resize(nc);
    for (int e = 0; e < n_edges; ++e) base_w[e] = p->edge_stiffness[e];
    for (int b = 0; b < n_bend; ++b) base_w[n_edges + b] = p->bend_weight;
    if (!finite_all(base_w.data(), nc)) { error = "non-finite weights"; return SIM_ENONFINITE; }
    for (double v : base_w)
        if (v < 0) { error = "weights must be >= 0"; return SIM_EINVAL; }
    region.clear();
    region_scale.clear();
    if (p->region_scale && p->n_regions > 0) {
        if (!p->edge_region || !p->bend_region) { error = "regions need edge_region and bend_region"; return SIM_EINVAL; }
        region_scale.assign(p->region_scale, p->region_scale + p->n_regions);
        if (!finite_all(region_scale.data(), region_scale.size())) { error = "non-finite region scale"; return SIM_ENONFINITE; }
        for (double v : region_scale)
            if (v < 0) { error = "region scales must be >= 0"; return SIM_EINVAL; }
        region.resize(nc);
        for (int e = 0; e < n_edges; ++e) region[e] = p->edge_region[e];
        for (int b = 0; b < n_bend; ++b) region[n_edges + b] = p->bend_region[bend_center[b]];
        for (int c = 0; c < nc; ++c)
            if (region[c] < 0 || region[c] >= p->n_regions) { error = "region index out of range"; return SIM_EINVAL; }
    }
    apply_regions();
    // rest norms and directions; flat bending (|l(X)| <= 1e-10 sum_k |c_k||X_k - X_b|) has no target
    rho.assign(nc, 0.0);
    restdir.assign(3 * (size_t)nc, 0.0);
    for (int c = 0; c < nc; ++c) {
        double q[3] = {0, 0, 0}, mag = 0;
        int ctr = c >= n_edges ? bend_center[c - n_edges] : -1;
        for (int k = c_ptr[c]; k < c_ptr[c + 1]; ++k) {
            const double *xk = &X[3 * c_node[k]];
            for (int d = 0; d < 3; ++d) q[d] += c_coef[k] * xk[d];
            if (ctr >= 0) {
                double dd[3];
                sub3(xk, &X[3 * ctr], dd);
                mag += std::fabs(c_coef[k]) * norm3(dd);
            }
        }
        double nq = norm3(q);
        if (ctr >= 0 && nq <= 1e-10 * mag) nq = 0.0;
        rho[c] = nq;
        if (nq > 0)
            for (int d = 0; d < 3; ++d) restdir[3 * c + d] = q[d] / nq;
    }
    // attachments
    attach.assign(mesh->attach, mesh->attach + mesh->n_attach);
    for (int a : attach)
        if (a < 0 || a >= m) { error = "attachment index out of range"; return SIM_EINVAL; }
    w_att = p->attach_weight;
    att_omega = mesh->attach_omega;
    for (int d = 0; d < 3; ++d) { att_axis[d] = mesh->attach_axis[d]; att_center[d] = mesh->attach_center[d]; }
    if (!attach.empty()) {
        double an = norm3(att_axis);
        if (!(an > 0)) { error = "attachment axis is zero"; return SIM_EINVAL; }
        for (int d = 0; d < 3; ++d) att_axis[d] /= an;
    }

    return assemble_ks(false);
}

// Effective constraint weights: base weight times its region scale (if any).
void HostModel::apply_regions() {
    w = base_w;
    if (!region.empty())
        for (int c = 0; c < nc; ++c) w[c] = base_w[c] * region_scale[region[c]];
}

// K_s = sum_c w_c a_c a_c^T + w_att sum_att e_j e_j^T.  The first call fixes
// the sparsity pattern (exact zeros off the diagonal dropped); later calls
// (keep_pattern) refill the values on that pattern and fail if a nonzero
// falls outside it.
int HostModel::assemble_ks(bool keep_pattern) {
    std::vector<std::map<int, double>> rows(m);
    for (int c = 0; c < nc; ++c) {
        for (int k = c_ptr[c]; k < c_ptr[c + 1]; ++k)
            for (int l = c_ptr[c]; l < c_ptr[c + 1]; ++l)
                rows[c_node[k]][c_node[l]] += w[c] * c_coef[k] * c_coef[l];
    }
    for (int a : attach) rows[a][a] += w_att;
    for (int i = 0; i < m; ++i) rows[i][i] += 0.0;   // keep the diagonal in the pattern
    if (keep_pattern) {
        std::vector<double> val(ks_col.size(), 0.0);
        for (int i = 0; i < m; ++i) {
            for (auto &kv : rows[i]) {
                const auto b = ks_col.begin() + ks_ptr[i], e = ks_col.begin() + ks_ptr[i + 1];
                const auto it = std::lower_bound(b, e, kv.first);
                if (it == e || *it != kv.first) {
                    if (kv.second == 0.0) continue;
                    error = "the new weights change the sparsity pattern of K";
                    return SIM_EINVAL;
                }
                val[it - ks_col.begin()] = kv.second;
            }
        }
        ks_val.swap(val);
        return SIM_OK;
    }
    ks_ptr.assign(1, 0);
    ks_col.clear();
    ks_val.clear();
    for (int i = 0; i < m; ++i) {
        for (auto &kv : rows[i]) {
            if (kv.second == 0.0 && kv.first != i) continue;
            ks_col.push_back(kv.first);
            ks_val.push_back(kv.second);
        }
        ks_ptr.push_back((int32_t)ks_col.size());
    }
    return SIM_OK;
}

// --------------------------------------------------------------------------
// Nested dissection: split a node set at the median of its longest rest-shape
// extent, take the smaller one-sided boundary of the cut as the separator
// (this also separates the bending 2-ring couplings), recurse on both sides,
// and number the separator last.  Leaves of <= leaf_size nodes and the
// separators become the (relaxed, dense) supernodes.
// --------------------------------------------------------------------------
namespace {

struct NDCtx {
    const std::vector<int32_t> *ptr, *col;
    const std::vector<double> *X;
    int leaf;
    std::vector<int32_t> order;        // new -> old
    std::vector<int32_t> sup_sizes;    // block sizes in elimination order (post-order)
    std::vector<int32_t> sep_depth;    // per block: depth of a separator, -1 for a leaf
    std::vector<int32_t> mark;         // scratch: 0 outside, 1 side A, 2 side B
};

void nd_rec(NDCtx &c, std::vector<int32_t> nodes, int depth) {
    const int n = (int)nodes.size();
    if (n == 0) return;
    if (n <= c.leaf) {
        std::sort(nodes.begin(), nodes.end());
        for (int v : nodes) c.order.push_back(v);
        c.sup_sizes.push_back(n);
        c.sep_depth.push_back(-1);
        return;
    }
    const auto &X = *c.X;
    std::vector<int32_t> best_sep, best_A, best_B;
    bool found = false;
    for (int ax = 0; ax < 3; ++ax) {
        std::vector<int32_t> sorted = nodes;
        std::stable_sort(sorted.begin(), sorted.end(), [&](int a, int b) {
            if (X[3 * a + ax] != X[3 * b + ax]) return X[3 * a + ax] < X[3 * b + ax];
            return a < b;
        });
        const int half = n / 2;
        for (int i = 0; i < n; ++i) c.mark[sorted[i]] = i < half ? 1 : 2;
        std::vector<int32_t> bA, bB;
        for (int v : nodes) {
            bool cross = false;
            for (int k = (*c.ptr)[v]; k < (*c.ptr)[v + 1]; ++k) {
                int u = (*c.col)[k];
                if (c.mark[u] != 0 && c.mark[u] != c.mark[v]) { cross = true; break; }
            }
            if (cross) (c.mark[v] == 1 ? bA : bB).push_back(v);
        }
        std::vector<int32_t> &sep = bA.size() <= bB.size() ? bA : bB;
        for (int v : sep) c.mark[v] = 3;
        std::vector<int32_t> A, B;
        for (int v : nodes) {
            if (c.mark[v] == 1) A.push_back(v);
            else if (c.mark[v] == 2) B.push_back(v);
        }
        for (int v : nodes) c.mark[v] = 0;
        if (A.empty() || B.empty() || sep.size() * 2 >= (size_t)n) continue;
        if (!found || sep.size() < best_sep.size()) {
            found = true;
            best_sep = sep;
            best_A = std::move(A);
            best_B = std::move(B);
        }
    }
    if (!found) {                                   // no useful cut
        std::sort(nodes.begin(), nodes.end());
        for (int v : nodes) c.order.push_back(v);
        c.sup_sizes.push_back(n);
        c.sep_depth.push_back(-1);
        return;
    }
    std::vector<int32_t> &sep = best_sep, &A = best_A, &B = best_B;
    nd_rec(c, A, depth + 1);
    nd_rec(c, B, depth + 1);
    std::sort(sep.begin(), sep.end());
    for (int v : sep) c.order.push_back(v);
    c.sup_sizes.push_back((int)sep.size());
    c.sep_depth.push_back(depth);
}

// Supernodal structure of a partition of the columns (in elimination order)
// into consecutive blocks c0[0] < c0[1] < ...: the off-diagonal rows R_s of
// every block (its own couplings past its last column plus the rows passed up
// by its children) and the levels of the resulting tree.
void symbolic(const std::vector<std::vector<int32_t>> &adj, const std::vector<int32_t> &c0,
              std::vector<int32_t> &R_ptr, std::vector<int32_t> &R_rows, std::vector<int32_t> &level, int &n_levels) {
    const int ns = (int)c0.size() - 1, m = (int)adj.size();
    std::vector<int32_t> blk(m);
    for (int s = 0; s < ns; ++s)
        for (int c = c0[s]; c < c0[s + 1]; ++c) blk[c] = s;
    std::vector<std::vector<int32_t>> pend(ns);
    std::vector<int32_t> parent(ns, -1);
    std::vector<char> seen(m, 0);
    R_ptr.assign(1, 0);
    R_rows.clear();
    for (int s = 0; s < ns; ++s) {
        const int a = c0[s], b = c0[s + 1];
        std::vector<int32_t> rs;
        auto add = [&](int r) {
            if (r >= b && !seen[r]) { seen[r] = 1; rs.push_back(r); }
        };
        for (int c = a; c < b; ++c)
            for (int r : adj[c]) add(r);
        for (int r : pend[s]) add(r);
        for (int r : rs) seen[r] = 0;
        std::sort(rs.begin(), rs.end());
        if (!rs.empty()) {
            const int p = blk[rs[0]];
            parent[s] = p;
            pend[p].insert(pend[p].end(), rs.begin(), rs.end());
        }
        R_rows.insert(R_rows.end(), rs.begin(), rs.end());
        R_ptr.push_back((int32_t)R_rows.size());
        pend[s].clear();
        pend[s].shrink_to_fit();
    }
    level.assign(ns, 0);
    n_levels = 0;
    for (int s = 0; s < ns; ++s) {                       // children precede parents
        if (parent[s] >= 0) level[parent[s]] = std::max(level[parent[s]], level[s] + 1);
        n_levels = std::max(n_levels, level[s] + 1);
    }
}

}  // namespace

int HostModel::order_and_factor(int leaf_size, int merge_cap) {
    order(leaf_size, merge_cap);
    return factor();
}

// Nested dissection, then: the separators of the top levels of the dissection
// tree (as many levels as keep their total at most merge_cap nodes) are
// numbered last, in post-order.  For the factor of P they form one dense
// supernode (one level of the solves instead of several short ones); the
// direct adjoint keeps them as separate supernodes and cuts every supernode
// into chunks of at most lu_chunk nodes.
void HostModel::order(int leaf_size, int merge_cap) {
    NDCtx ctx;
    ctx.ptr = &ks_ptr;
    ctx.col = &ks_col;
    ctx.X = &X;
    ctx.leaf = std::max(4, leaf_size);
    ctx.mark.assign(m, 0);
    std::vector<int32_t> all(m);
    std::iota(all.begin(), all.end(), 0);
    nd_rec(ctx, all, 0);
    const int nb = (int)ctx.sup_sizes.size();
    int merge_depth = 0;
    for (int d = 1;; ++d) {
        int tot = 0, cnt = 0, deeper = 0;
        for (int b = 0; b < nb; ++b) {
            if (ctx.sep_depth[b] >= 0 && ctx.sep_depth[b] < d) { tot += ctx.sup_sizes[b]; ++cnt; }
            if (ctx.sep_depth[b] >= d) ++deeper;
        }
        if (tot > merge_cap || cnt == 0) break;
        merge_depth = d;
        if (!deeper) break;
    }
    if (merge_depth < 2) merge_depth = 0;              // merging one separator changes nothing
    // final order: blocks in post-order, the merged separators moved to the end
    std::vector<int32_t> bstart(nb + 1, 0);
    for (int b = 0; b < nb; ++b) bstart[b + 1] = bstart[b] + ctx.sup_sizes[b];
    auto merged = [&](int b) { return ctx.sep_depth[b] >= 0 && ctx.sep_depth[b] < merge_depth; };
    perm.clear();
    std::vector<int32_t> psizes, lsizes;                 // P's blocks, the adjoint's blocks
    for (int b = 0; b < nb; ++b)
        if (!merged(b)) {
            perm.insert(perm.end(), ctx.order.begin() + bstart[b], ctx.order.begin() + bstart[b + 1]);
            psizes.push_back(ctx.sup_sizes[b]);
            lsizes.push_back(ctx.sup_sizes[b]);
        }
    int mtot = 0;
    for (int b = 0; b < nb; ++b)
        if (merged(b)) {
            perm.insert(perm.end(), ctx.order.begin() + bstart[b], ctx.order.begin() + bstart[b + 1]);
            lsizes.push_back(ctx.sup_sizes[b]);
            mtot += ctx.sup_sizes[b];
        }
    if (mtot) psizes.push_back(mtot);
    merged_nodes = mtot;
    iperm.assign(m, -1);
    for (int i = 0; i < m; ++i) iperm[perm[i]] = i;
    ns = (int)psizes.size();
    sup_c0.assign(ns + 1, 0);
    for (int s = 0; s < ns; ++s) sup_c0[s + 1] = sup_c0[s] + psizes[s];
    sup_of.assign(m, 0);
    for (int s = 0; s < ns; ++s)
        for (int c = sup_c0[s]; c < sup_c0[s + 1]; ++c) sup_of[c] = s;
    lu_c0.assign(1, 0);
    for (int sz : lsizes) {
        const int nck = (sz + lu_chunk - 1) / lu_chunk, base = lu_c0.back();
        for (int j = 1; j <= nck; ++j) lu_c0.push_back(base + (int)((int64_t)sz * j / nck));
    }

    // permuted lower pattern: for new column c, rows r > c adjacent to it
    std::vector<std::vector<int32_t>> adj(m);
    for (int oi = 0; oi < m; ++oi) {
        int ci = iperm[oi];
        for (int k = ks_ptr[oi]; k < ks_ptr[oi + 1]; ++k) {
            int rj = iperm[ks_col[k]];
            if (rj > ci) adj[ci].push_back(rj);
        }
    }
    symbolic(adj, sup_c0, R_ptr, R_rows, sup_level, n_levels);
    symbolic(adj, lu_c0, lu_R_ptr, lu_R_rows, lu_level, lu_n_levels);
}

// Numeric factorisation on the symbolic structure of order() (left-looking,
// dense blocks); refactoring after a weight change reuses the structure.
int HostModel::factor() {
    std::vector<std::vector<int32_t>> R(ns);
    for (int s = 0; s < ns; ++s) R[s].assign(R_rows.begin() + R_ptr[s], R_rows.begin() + R_ptr[s + 1]);
    Lblk.assign(ns, {});
    std::vector<std::vector<int32_t>> updaters(ns);
    std::vector<int32_t> rowpos(m, -1);
    nnz_L = 0;
    const double hh = h * h;
    for (int s = 0; s < ns; ++s) {
        const int c0 = sup_c0[s], c1 = sup_c0[s + 1], nsc = c1 - c0;
        const int nR = (int)R[s].size(), nrow = nsc + nR;
        std::vector<double> &F = Lblk[s];
        F.assign((size_t)nrow * nsc, 0.0);
        for (int c = c0; c < c1; ++c) rowpos[c] = c - c0;
        for (int i = 0; i < nR; ++i) rowpos[R[s][i]] = nsc + i;
        // assemble P_s columns c0..c1-1 (lower part)
        for (int c = c0; c < c1; ++c) {
            int oc = perm[c];
            for (int k = ks_ptr[oc]; k < ks_ptr[oc + 1]; ++k) {
                int r = iperm[ks_col[k]];
                if (r < c) continue;
                double v = hh * ks_val[k] + (r == c ? mass[oc] : 0.0);
                F[(size_t)(c - c0) * nrow + rowpos[r]] += v;
            }
        }
        // updates from descendants
        for (int d : updaters[s]) {
            const auto &Rd = R[d];
            const int nsd = sup_c0[d + 1] - sup_c0[d], nrd = nsd + (int)Rd.size();
            const auto &Ld = Lblk[d];
            int i0 = (int)(std::lower_bound(Rd.begin(), Rd.end(), c0) - Rd.begin());
            int i1 = (int)(std::lower_bound(Rd.begin(), Rd.end(), c1) - Rd.begin());
            for (int j = i0; j < i1; ++j) {
                const int colloc = Rd[j] - c0;
                for (int i = j; i < (int)Rd.size(); ++i) {
                    double acc = 0;
                    for (int k = 0; k < nsd; ++k)
                        acc += Ld[(size_t)k * nrd + nsd + i] * Ld[(size_t)k * nrd + nsd + j];
                    F[(size_t)colloc * nrow + rowpos[Rd[i]]] -= acc;
                }
            }
        }
        // dense Cholesky of the diagonal block, then the off-diagonal rows
        for (int k = 0; k < nsc; ++k) {
            double dkk = F[(size_t)k * nrow + k];
            for (int l = 0; l < k; ++l) dkk -= F[(size_t)l * nrow + k] * F[(size_t)l * nrow + k];
            if (!(dkk > 0) || !std::isfinite(dkk)) {
                error = "P is not positive definite";
                return SIM_ENOTSPD;
            }
            const double lkk = std::sqrt(dkk);
            F[(size_t)k * nrow + k] = lkk;
            for (int i = k + 1; i < nrow; ++i) {
                double v = F[(size_t)k * nrow + i];
                for (int l = 0; l < k; ++l) v -= F[(size_t)l * nrow + i] * F[(size_t)l * nrow + k];
                F[(size_t)k * nrow + i] = v / lkk;
            }
        }
        for (int k = 0; k < nsc; ++k)
            for (int i = 0; i < k; ++i) F[(size_t)k * nrow + i] = 0.0;
        nnz_L += (int64_t)nsc * (nsc + 1) / 2 + (int64_t)nR * nsc;
        for (int c = c0; c < c1; ++c) rowpos[c] = -1;
        for (int i = 0; i < nR; ++i) rowpos[R[s][i]] = -1;
        // register s as an updater of the supernodes its rows fall in
        int last = -1;
        for (int r : R[s]) {
            int t = sup_of[r];
            if (t != last) { updaters[t].push_back(s); last = t; }
        }
    }
    return SIM_OK;
}

void HostModel::dense_L(double *out) const {
    std::fill(out, out + (size_t)m * m, 0.0);
    for (int s = 0; s < ns; ++s) {
        const int c0 = sup_c0[s], nsc = sup_c0[s + 1] - c0;
        const int nR = R_ptr[s + 1] - R_ptr[s], nrow = nsc + nR;
        for (int k = 0; k < nsc; ++k) {
            for (int i = k; i < nsc; ++i) out[(size_t)(c0 + i) * m + c0 + k] = Lblk[s][(size_t)k * nrow + i];
            for (int i = 0; i < nR; ++i)
                out[(size_t)R_rows[R_ptr[s] + i] * m + c0 + k] = Lblk[s][(size_t)k * nrow + nsc + i];
        }
    }
}

}  // namespace dc
