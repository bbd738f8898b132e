// gfx950 kernels of the DiffCloth hot path.
//
// One workgroup of 1024 threads (16 wavefronts) owns one cloth handle for a
// whole launch: it runs every time step of a forward segment (PD local/global
// iterations with the contact update) or every adjoint step of a backward
// segment without returning to the host.  A batched launch gives each handle
// its own workgroup.  All vectors stay in HBM / L2; workgroup barriers order
// the phases, so results do not depend on scheduling (no floating-point
// atomics anywhere: every sum has a fixed order).
#include <hip/hip_runtime.h>
#include <type_traits>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "sim_dev.h"

namespace dc {

// Pointers read from the descriptor are HBM (global) pointers; saying so lets
// the compiler emit global (not flat) memory instructions, so loads to HBM and
// LDS are tracked by separate counters and overlap.
#define GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GLOBAL T *G(T *p) { return (GLOBAL T *)p; }
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v2i __attribute__((ext_vector_type(2)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
// compile-time choice between an LDS and an HBM pointer (their types differ)
template <bool C, class P, class Q>
__device__ __forceinline__ auto pick(P a, Q b) {
    if constexpr (C) return a;
    else return b;
}

constexpr uint8_t FREE = 0, TAKEOFF = 1, STICK = 2, SLIP = 3;

// ------------------------------------------------------------------ reductions

__device__ inline double team_sum(double v, int tl) {
    for (int o = tl >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, tl);
    return v;
}

// Block-wide max of a non-negative value; every thread gets the result.
__device__ inline double block_max(double v, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, red[w]);
    return r;
}

// Block-wide sum in a fixed order (wave butterflies, then waves 0..15).
__device__ inline double block_sum(double v, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r += red[w];
    return r;
}

// ------------------------------------------------------------------ global solve
// P v = b with P = P_s (x) I_3 = (L L^T) (x) I_3, three right-hand sides held
// node-major.  Supernodes of one level of the elimination tree are independent.
// Each supernode s stores G_s = [L_ss^{-1}; B_s L_ss^{-1}] (column-major), so
//   forward,  per level: (1) t_i = b_i - sum of the update entries of descendant
//             supernodes that reach row i; (2) [y_s; u_s] = G_s t_s;
//   backward, per level: x_s = L_ss^{-T} y_s - (B_s L_ss^{-1})^T x_{R_s}.
// Work items are packed descriptors; the host picks the lanes per item of each
// level.  T, Y and the update buffer U live in LDS when they fit.  b may alias
// T; x may alias T (T is dead once a level's products are formed).
// Forward-solve gather of one level: t_i = b_i - (the update entries reaching
// row i, in list order), a row per thread; four update offsets and their
// entries are loaded before the subtractions.
__device__ __forceinline__ void gather_rows(GLOBAL const RowItem *rows, GLOBAL const int32_t *upd, int r0, int r1,
                                            auto b, auto T, auto U) {
    for (int t = r0 + (int)threadIdx.x; t < r1; t += (int)blockDim.x) {
        const auto &it = rows[t];
        const int i3 = it.i3, p1 = it.p1;
        double a0 = b[i3], a1 = b[i3 + 1], a2 = b[i3 + 2];
        int p = it.p0;
        for (; p + 4 <= p1; p += 4) {
            int o[4];
            double u[4][3];
#pragma unroll
            for (int j = 0; j < 4; ++j) o[j] = upd[p + j];
#pragma unroll
            for (int j = 0; j < 4; ++j) { u[j][0] = U[o[j]]; u[j][1] = U[o[j] + 1]; u[j][2] = U[o[j] + 2]; }
#pragma unroll
            for (int j = 0; j < 4; ++j) { a0 -= u[j][0]; a1 -= u[j][1]; a2 -= u[j][2]; }
        }
        for (; p < p1; ++p) {
            const int o = upd[p];
            a0 -= U[o]; a1 -= U[o + 1]; a2 -= U[o + 2];
        }
        T[i3] = a0; T[i3 + 1] = a1; T[i3 + 2] = a2;
    }
}

// Writes the forward-solve result of one row: Y (diagonal-block rows) or the
// update buffer (rows of B_s), or nothing for a padding row.
__device__ __forceinline__ void put_row(int out, double a0, double a1, double a2, auto Y, auto U) {
    if (out >= 0) {
        Y[out] = a0; Y[out + 1] = a1; Y[out + 2] = a2;
    } else if (out != kNoOutput) {
        const int o = -out - 1;
        U[o] = a0; U[o + 1] = a1; U[o + 2] = a2;
    }
}

constexpr int64_t kPosMask = (int64_t(1) << 40) - 1;      // position bits of adj_pos / fwd_pos

// thread 0 announces a position (epoch << 40 | pos) to prefetch workgroups
__device__ __forceinline__ void announce(int64_t *where, int64_t epoch, int64_t pos) {
    if (threadIdx.x == 0) __hip_atomic_store(where, (epoch << 40) | pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Forward-solve products of items t0, t0 + stride, ... < t1 (rows r, r + 1 of a
// stacked block G_s times the gathered right-hand side), one team of tl lanes
// per item; cur / cur2 hold the first item's descriptor (fetched early by the
// caller), the next one is in flight while the current one is computed.
// Whole batches of a lane's columns run without bounds checks, the last,
// partial one with them; the columns are taken in the same order either way.
__device__ __forceinline__ void fwd_products(GLOBAL const v4i *fit, auto gv2, int t0, int t1, int stride,
                                             int tl, int lane, v4i cur, v4i cur2, auto T, auto Y, auto U) {
    for (int t = t0; t < t1; t += stride) {
        v4i nxt = {0, 0, 0, 0}, nxt2 = {0, 0, 0, 0};  // next descriptor, in flight meanwhile
        if (t + stride < t1) { nxt = fit[2 * (t + stride)]; nxt2 = fit[2 * (t + stride) + 1]; }
        const auto Gb = gv2 + (cur.x >> 1);
        const auto Tb = T + cur.z;
        const int ld2 = (cur.y & 0xffff) >> 1, kmax = cur.y >> 16;
        double a0 = 0, a1 = 0, a2 = 0, b0 = 0, b1 = 0, b2 = 0;
        auto acc = [&](v2d g, int k) {
            const double t0v = Tb[3 * k], t1v = Tb[3 * k + 1], t2v = Tb[3 * k + 2];
            a0 += g.x * t0v; a1 += g.x * t1v; a2 += g.x * t2v;
            b0 += g.y * t0v; b1 += g.y * t1v; b2 += g.y * t2v;
        };
        const int step = kSolveBatch * tl;
        int k0 = lane;
        for (; k0 + (kSolveBatch - 1) * tl < kmax; k0 += step) {
            v2d g[kSolveBatch];
#pragma unroll
            for (int j = 0; j < kSolveBatch; ++j) g[j] = Gb[(k0 + j * tl) * ld2];   // loads in flight together
#pragma unroll
            for (int j = 0; j < kSolveBatch; ++j) acc(g[j], k0 + j * tl);
        }
        if (k0 < kmax) {
            v2d g[kSolveBatch];
#pragma unroll
            for (int j = 0; j < kSolveBatch; ++j) {
                const int k = k0 + j * tl;
                g[j] = k < kmax ? Gb[k * ld2] : v2d{0.0, 0.0};
            }
#pragma unroll
            for (int j = 0; j < kSolveBatch; ++j)
                if (k0 + j * tl < kmax) acc(g[j], k0 + j * tl);
        }
        a0 = team_sum(a0, tl); a1 = team_sum(a1, tl); a2 = team_sum(a2, tl);
        b0 = team_sum(b0, tl); b1 = team_sum(b1, tl); b2 = team_sum(b2, tl);
        if (lane == 0) {
            put_row(cur.w, a0, a1, a2, Y, U);
            put_row(cur2.x, b0, b1, b2, Y, U);
        }
        cur = nxt;
        cur2 = nxt2;
    }
}

// Backward-solve products of items t0, t0 + stride, ... < t1 (column pairs of
// a stacked block: x_s = L_ss^{-T} y_s - (B_s L_ss^{-1})^T x_{R_s}, x_{R_s}
// gathered into the supernode's update slots first).  A lane's rows of the
// diagonal block come first, then those of B_s; whole batches on either side
// run without bounds checks, in the same order as the checked batches.
__device__ __forceinline__ void bwd_products(GLOBAL const v4i *bit, GLOBAL const v2d *gt2, int t0, int t1, int stride,
                                             int tl, int lane, v4i cur, v4i cur2, auto Y, auto x, auto U) {
    for (int t = t0; t < t1; t += stride) {
        v4i nxt = {0, 0, 0, 0}, nxt2 = {0, 0, 0, 0};
        if (t + stride < t1) { nxt = bit[2 * (t + stride)]; nxt2 = bit[2 * (t + stride) + 1]; }
        const auto Gb = gt2 + (cur.x >> 1);
        const int st2 = cur2.x >> 1;
        const int n1 = cur.y & 0xffff, n = n1 + (cur.y >> 16), yb = cur.z;
        const auto Yb = Y + yb;
        const int ub = cur.w - 3 * n1;               // U[ub + 3k] is row k >= n1
        double a0 = 0, a1 = 0, a2 = 0, b0 = 0, b1 = 0, b2 = 0;
        auto acc_y = [&](v2d g, int k) {                 // row k < n1: times y_s
            const double w0 = Yb[3 * k], w1 = Yb[3 * k + 1], w2 = Yb[3 * k + 2];
            a0 += g.x * w0; a1 += g.x * w1; a2 += g.x * w2;
            b0 += g.y * w0; b1 += g.y * w1; b2 += g.y * w2;
        };
        auto acc_u = [&](v2d g, int k) {                 // row k >= n1: minus times x_{R_s}
            const int o = ub + 3 * k;
            const double w0 = U[o], w1 = U[o + 1], w2 = U[o + 2];
            a0 -= g.x * w0; a1 -= g.x * w1; a2 -= g.x * w2;
            b0 -= g.y * w0; b1 -= g.y * w1; b2 -= g.y * w2;
        };
        const int step = kSolveBatch * tl;
        int k0 = lane;
        for (; k0 + (kSolveBatch - 1) * tl < n1; k0 += step) {   // whole batches of y_s rows
            v2d g[kSolveBatch];
#pragma unroll
            for (int j = 0; j < kSolveBatch; ++j) g[j] = Gb[(k0 + j * tl) * st2];
#pragma unroll
            for (int j = 0; j < kSolveBatch; ++j) acc_y(g[j], k0 + j * tl);
        }
        if (k0 < n) {                                            // the batch reaching past n1 (checked)
            v2d g[kSolveBatch];
#pragma unroll
            for (int j = 0; j < kSolveBatch; ++j) {
                const int k = k0 + j * tl;
                g[j] = k < n ? Gb[k * st2] : v2d{0.0, 0.0};
            }
#pragma unroll
            for (int j = 0; j < kSolveBatch; ++j) {
                const int k = k0 + j * tl;
                if (k < n1) acc_y(g[j], k);
                else if (k < n) acc_u(g[j], k);
            }
            k0 += step;
        }
        for (; k0 + (kSolveBatch - 1) * tl < n; k0 += step) {    // whole batches of x_{R_s} rows
            v2d g[kSolveBatch];
#pragma unroll
            for (int j = 0; j < kSolveBatch; ++j) g[j] = Gb[(k0 + j * tl) * st2];
#pragma unroll
            for (int j = 0; j < kSolveBatch; ++j) acc_u(g[j], k0 + j * tl);
        }
        if (k0 < n) {                                            // the last, partial batch
            v2d g[kSolveBatch];
#pragma unroll
            for (int j = 0; j < kSolveBatch; ++j) {
                const int k = k0 + j * tl;
                g[j] = k < n ? Gb[k * st2] : v2d{0.0, 0.0};
            }
#pragma unroll
            for (int j = 0; j < kSolveBatch; ++j)
                if (k0 + j * tl < n) acc_u(g[j], k0 + j * tl);
        }
        a0 = team_sum(a0, tl); a1 = team_sum(a1, tl); a2 = team_sum(a2, tl);
        b0 = team_sum(b0, tl); b1 = team_sum(b1, tl); b2 = team_sum(b2, tl);
        if (lane == 0) {
            x[yb] = a0; x[yb + 1] = a1; x[yb + 2] = a2;
            if (cur2.y) { x[yb + 3] = b0; x[yb + 4] = b1; x[yb + 5] = b2; }
        }
        cur = nxt;
        cur2 = nxt2;
    }
}

// backward gathers q0 .. q1 - 1 (x_{R_s} into the update slots; a root's rows read from Y), from thread t
__device__ __forceinline__ void bwd_gather(GLOBAL const v2i *bg, int q0, int q1, int t, int nt, auto x, auto Y, auto U) {
    for (int q = q0 + t; q < q1; q += nt) {
        const v2i e = bg[q];                             // GatherItem {u, x3}
        if (e.y >= 0) {
            U[e.x] = x[e.y]; U[e.x + 1] = x[e.y + 1]; U[e.x + 2] = x[e.y + 2];
        } else {                                         // a root's row: x is still in Y
            const int y3 = -e.y - 1;
            U[e.x] = Y[y3]; U[e.x + 1] = Y[y3 + 1]; U[e.x + 2] = Y[y3 + 2];
        }
    }
}

// pos0 >= 0: the forward pass announces each level (pos0 + phase, see fwd_pos)
__device__ __forceinline__ void solve_P(const SimDev &S, GLOBAL const int32_t *team_of, auto b, auto T, auto Y, auto x, auto U,
                                        int64_t pos0 = -1) {
    const auto gv2 = (GLOBAL const v2d *)S.gval;        // two rows per load
    const auto gt2 = (GLOBAL const v2d *)S.gvalt;       // two columns per load
    for (int l = 0; l < S.n_levels; ++l) {
        if (pos0 >= 0) announce(S.fwd_pos, S.fwd_epoch, pos0 + l);
        // descriptor of this thread's first product item, fetched before the
        // gather phase and its barrier (it does not depend on the vectors)
        const int tl = team_of[2 * l];
        const int team = threadIdx.x / tl, lane = threadIdx.x % tl, nteams = (int)blockDim.x / tl;
        const int i0 = G(S.lvl_items_ptr)[l], i1 = G(S.lvl_items_ptr)[l + 1];
        const auto fit = (GLOBAL const v4i *)S.fitems;  // FwdItem as 2 x 16 bytes
        v4i cur = {0, 0, 0, 0}, cur2 = {0, 0, 0, 0};
        if (i0 + team < i1) { cur = fit[2 * (i0 + team)]; cur2 = fit[2 * (i0 + team) + 1]; }
        gather_rows(G(S.rows), G(S.upd_off), G(S.lvl_rows_ptr)[l], G(S.lvl_rows_ptr)[l + 1], b, T, U);
        __syncthreads();
        fwd_products(fit, gv2, i0 + team, i1, nteams, tl, lane, cur, cur2, T, Y, U);
        __syncthreads();
    }
    // backward: the update buffer is free; each level first gathers x_{R_s}
    // of its supernodes into their update slots, then forms
    // x_s = L_ss^{-T} y_s - (B_s L_ss^{-1})^T x_{R_s}, one item per column pair
    // of G_s (row-major copy: the items of a wavefront read consecutive addresses)
    for (int l = S.n_levels - 1; l >= 0; --l) {
        if (pos0 >= 0) announce(S.fwd_pos, S.fwd_epoch, pos0 + 2 * S.n_levels - 1 - l);
        const int tl = team_of[2 * l + 1];
        const int team = threadIdx.x / tl, lane = threadIdx.x % tl, nteams = (int)blockDim.x / tl;
        const int c0 = G(S.lvl_bwd_ptr)[l], c1 = G(S.lvl_bwd_ptr)[l + 1];
        const auto bit = (GLOBAL const v4i *)S.bitems;  // BwdItem as 2 x 16 bytes
        v4i cur = {0, 0, 0, 0}, cur2 = {0, 0, 0, 0};
        if (c0 + team < c1) { cur = bit[2 * (c0 + team)]; cur2 = bit[2 * (c0 + team) + 1]; }
        const int q0 = G(S.lvl_gat_ptr)[l], q1 = G(S.lvl_gat_ptr)[l + 1];
        if (c1 == c0 && q1 == q0 && l > 0) continue;    // root supernodes only: solved in the forward sweep
        if (q1 > q0) {
            bwd_gather((GLOBAL const v2i *)S.bgat, q0, q1, threadIdx.x, blockDim.x, x, Y, U);
            __syncthreads();
        }
        bwd_products(bit, gt2, c0 + team, c1, nteams, tl, lane, cur, cur2, Y, x, U);
        if (l == 0)                                      // the roots' x, left in Y by the forward sweep
            for (int q = threadIdx.x; q < S.n_root_rows; q += (int)blockDim.x) {
                const int i3 = G(S.root_rows)[q];
                x[i3] = Y[i3]; x[i3 + 1] = Y[i3 + 1]; x[i3 + 2] = Y[i3 + 2];
            }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ geometry

// Closest point of triangle T (a, b, c, unit face normal, bounding-ball
// centre and radius: 16 doubles) to x by Voronoi regions, following the
// published closest-point-on-triangle test of C. Ericson, Real-Time Collision
// Detection (2005), Sec. 5.1.5 (same region order and barycentric terms); returns the distance (plane distance on the face) and
// the region (0 face, 1 vertex, 2 edge).  WANT: also the closest point q, the
// edge vector ed (unnormalised) and the face distance fd.
template <bool WANT>
__device__ __forceinline__ double tri_closest(GLOBAL const double *T, const double *x, int &reg, double *q, double *ed,
                                              double &fd) {
#pragma clang fp contract(off)
    const double ab[3] = {T[3] - T[0], T[4] - T[1], T[5] - T[2]};
    const double ac[3] = {T[6] - T[0], T[7] - T[1], T[8] - T[2]};
    const double ap[3] = {x[0] - T[0], x[1] - T[1], x[2] - T[2]};
    const double bp[3] = {x[0] - T[3], x[1] - T[4], x[2] - T[5]};
    const double cp[3] = {x[0] - T[6], x[1] - T[7], x[2] - T[8]};
    const double d1 = ab[0] * ap[0] + ab[1] * ap[1] + ab[2] * ap[2];
    const double d2 = ac[0] * ap[0] + ac[1] * ap[1] + ac[2] * ap[2];
    const double d3 = ab[0] * bp[0] + ab[1] * bp[1] + ab[2] * bp[2];
    const double d4 = ac[0] * bp[0] + ac[1] * bp[1] + ac[2] * bp[2];
    const double d5 = ab[0] * cp[0] + ab[1] * cp[1] + ab[2] * cp[2];
    const double d6 = ac[0] * cp[0] + ac[1] * cp[1] + ac[2] * cp[2];
    const double vc = d1 * d4 - d3 * d2, vb = d5 * d2 - d1 * d6, va = d3 * d6 - d5 * d4;
    double r[3];                                     // x - q
    if (d1 <= 0 && d2 <= 0) {
        reg = 1;
        for (int d = 0; d < 3; ++d) r[d] = ap[d];
        if constexpr (WANT) for (int d = 0; d < 3; ++d) q[d] = T[d];
    } else if (d3 >= 0 && d4 <= d3) {
        reg = 1;
        for (int d = 0; d < 3; ++d) r[d] = bp[d];
        if constexpr (WANT) for (int d = 0; d < 3; ++d) q[d] = T[3 + d];
    } else if (vc <= 0 && d1 >= 0 && d3 <= 0) {
        reg = 2;
        const double v = d1 / (d1 - d3);
        double qq[3];
        for (int d = 0; d < 3; ++d) { qq[d] = T[d] + v * ab[d]; r[d] = x[d] - qq[d]; }
        if constexpr (WANT) for (int d = 0; d < 3; ++d) { q[d] = qq[d]; ed[d] = ab[d]; }
    } else if (d6 >= 0 && d5 <= d6) {
        reg = 1;
        for (int d = 0; d < 3; ++d) r[d] = cp[d];
        if constexpr (WANT) for (int d = 0; d < 3; ++d) q[d] = T[6 + d];
    } else if (vb <= 0 && d2 >= 0 && d6 <= 0) {
        reg = 2;
        const double w = d2 / (d2 - d6);
        double qq[3];
        for (int d = 0; d < 3; ++d) { qq[d] = T[d] + w * ac[d]; r[d] = x[d] - qq[d]; }
        if constexpr (WANT) for (int d = 0; d < 3; ++d) { q[d] = qq[d]; ed[d] = ac[d]; }
    } else if (va <= 0 && d4 - d3 >= 0 && d5 - d6 >= 0) {
        reg = 2;
        const double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        double qq[3];
        for (int d = 0; d < 3; ++d) { qq[d] = T[3 + d] + w * (T[6 + d] - T[3 + d]); r[d] = x[d] - qq[d]; }
        if constexpr (WANT) for (int d = 0; d < 3; ++d) { q[d] = qq[d]; ed[d] = T[6 + d] - T[3 + d]; }
    } else {
        reg = 0;
        r[0] = r[1] = r[2] = 0.0;
    }
    const double f = T[9] * ap[0] + T[10] * ap[1] + T[11] * ap[2];
    if constexpr (WANT) fd = f;
    return reg == 0 ? fabs(f) : sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
}

// Frame of a triangle-mesh obstacle at x: the closest triangle (ties to the
// lowest index; a first sweep bounds the distance by the nearest centroid c_t,
// a point of the mesh, and the exact test runs only where the triangle's ball
// can reach that bound, |x - c_t| - r_t <= bound; both sweeps in float with
// margins), then
// its closest point by Voronoi regions (tested in the order vertex a, vertex
// b, edge ab, vertex c, edge ac, edge bc, face).  Face: n = the face normal,
// phi = n.(x - a).  Edge or vertex with closest point q: r = |x - q|, s = the
// side of the face, phi = s r, n = s (x - q) / r (the face normal when r = 0).
// region: 0 face, 1 vertex, 2 edge, whose unit direction goes to e.  The
// arithmetic is unfused, in the written order: a node resting on a face has
// phi = 0 exactly, and the contact test phi <= 0 must come out the same in any
// implementation that evaluates these formulas as written.
__device__ __forceinline__ void mesh_frame(const ObstacleDev &ob, const double *x, double *n, double &phi, int &region,
                                           double *e) {
#pragma clang fp contract(off)
    const auto tri = (GLOBAL const double *)ob.tri;
    const auto b32 = (GLOBAL const v4f *)ob.ball32;
    // culling in float: coordinates of order metres round by < 1e-7 m, so the
    // bounds carry a margin of 1e-6 m (a looser cull, never a wrong one)
    constexpr float kCullMargin = 1e-6f;
    const float xf0 = (float)x[0], xf1 = (float)x[1], xf2 = (float)x[2];
    float ub2 = INFINITY;                            // the centroids lie on the mesh: min |x - c_t|
    for (int t = 0; t < ob.n_tris; ++t) {            // bounds the distance from above
        const v4f B = b32[t];
        const float c0 = xf0 - B.x, c1 = xf1 - B.y, c2 = xf2 - B.z;
        ub2 = fminf(ub2, c0 * c0 + c1 * c1 + c2 * c2);
    }
    const float ub = sqrtf(ub2) * (1.0f + 1e-6f) + 2.0f * kCullMargin;
    double best = INFINITY;
    int bt = 0;
    for (int t = 0; t < ob.n_tris; ++t) {
        const v4f B = b32[t];
        const float c0 = xf0 - B.x, c1 = xf1 - B.y, c2 = xf2 - B.z;
        const float reach = ub + B.w + kCullMargin;
        if (c0 * c0 + c1 * c1 + c2 * c2 > reach * reach * (1.0f + 1e-6f)) continue;   // |x - c_t| - r_t > ub
        int reg;
        double fd;
        const double dist = tri_closest<false>(tri + 16 * (int64_t)t, x, reg, nullptr, nullptr, fd);
        if (dist < best) { best = dist; bt = t; }
    }
    const auto T = tri + 16 * (int64_t)bt;
    double q[3] = {0.0, 0.0, 0.0}, ed[3] = {0.0, 0.0, 0.0}, fd;
    int breg;
    (void)tri_closest<true>(T, x, breg, q, ed, fd);
    const double bn[3] = {T[9], T[10], T[11]};
    region = breg;
    e[0] = e[1] = e[2] = 0.0;
    if (breg == 0) {
        phi = fd;
        for (int d = 0; d < 3; ++d) n[d] = bn[d];
        return;
    }
    const double r0 = x[0] - q[0], r1 = x[1] - q[1], r2 = x[2] - q[2];
    const double r = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
    const double sg = (bn[0] * r0 + bn[1] * r1 + bn[2] * r2 >= 0.0) ? 1.0 : -1.0;
    if (r > 0.0) {
        phi = sg * r;
        n[0] = sg * r0 / r; n[1] = sg * r1 / r; n[2] = sg * r2 / r;
    } else {
        phi = 0.0;
        for (int d = 0; d < 3; ++d) n[d] = bn[d];
    }
    if (breg == 2) {
        const double le = sqrt(ed[0] * ed[0] + ed[1] * ed[1] + ed[2] * ed[2]);
        for (int d = 0; d < 3; ++d) e[d] = ed[d] / le;
    }
}

template <bool MESH = true>
__device__ __forceinline__ void contact_frame(const SimDev &S, int o, auto xi, double *n, double &phi) {
    const ObstacleDev &ob = S.obst[o];
    if constexpr (MESH) {
        if (ob.type == 2) {
            const double x[3] = {xi[0], xi[1], xi[2]};
            int reg;
            double e[3];
            mesh_frame(ob, x, n, phi, reg, e);
            return;
        }
    }
    if (ob.type == 0) {
        n[0] = ob.n[0]; n[1] = ob.n[1]; n[2] = ob.n[2];
        phi = (xi[0] - ob.p[0]) * n[0] + (xi[1] - ob.p[1]) * n[1] + (xi[2] - ob.p[2]) * n[2];
    } else {
        const double d0 = xi[0] - ob.p[0], d1 = xi[1] - ob.p[1], d2 = xi[2] - ob.p[2];
        const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        n[0] = d0 / r; n[1] = d1 / r; n[2] = d2 / r;
        phi = r - ob.radius;
    }
}

template <bool MESH>
__device__ __forceinline__ double signed_distance(const ObstacleDev &ob, const double *y) {
    if constexpr (MESH) {
        if (ob.type == 2) {
            if (ob.closed) {
                // outside a ball around a closed surface: outside the surface, and
                // phi > 0 is all the contact test needs (not its value)
                const double b0 = y[0] - ob.ball[0], b1 = y[1] - ob.ball[1], b2 = y[2] - ob.ball[2];
                const double db = sqrt(b0 * b0 + b1 * b1 + b2 * b2);
                if (db > ob.ball[3]) return db - ob.ball[3];
            }
            double n[3], phi, e[3];
            int reg;
            mesh_frame(ob, y, n, phi, reg, e);
            return phi;
        }
    }
    if (ob.type == 0)
        return (y[0] - ob.p[0]) * ob.n[0] + (y[1] - ob.p[1]) * ob.n[1] + (y[2] - ob.p[2]) * ob.n[2];
    const double d0 = y[0] - ob.p[0], d1 = y[1] - ob.p[1], d2 = y[2] - ob.p[2];
    return sqrt(d0 * d0 + d1 * d1 + d2 * d2) - ob.radius;
}

// attachment target of rest point X at time t: c + R(axis, omega t)(X - c)
__device__ __forceinline__ void attach_target(const SimDev &S, auto X, double t, double *out) {
    const double ang = S.att_omega * t, cs = cos(ang), sn = sin(ang);
    const double *a = S.att_axis;
    const double d0 = X[0] - S.att_center[0], d1 = X[1] - S.att_center[1], d2 = X[2] - S.att_center[2];
    const double ad = a[0] * d0 + a[1] * d1 + a[2] * d2;
    const double c0 = a[1] * d2 - a[2] * d1, c1 = a[2] * d0 - a[0] * d2, c2 = a[0] * d1 - a[1] * d0;
    out[0] = S.att_center[0] + d0 * cs + c0 * sn + a[0] * ad * (1 - cs);
    out[1] = S.att_center[1] + d1 * cs + c1 * sn + a[1] * ad * (1 - cs);
    out[2] = S.att_center[2] + d2 * cs + c2 * sn + a[2] * ad * (1 - cs);
}

// Closed-form Signorini-Coulomb update of one node with isotropic response
// v = ub + f/m; gap-corrected normal velocity.  Decisions in float64.
__device__ __forceinline__ uint8_t signorini_coulomb(const double *ub, const double *n, double phi, double mu,
                                            double h, double mass, double *v, double *f) {
    const double un = n[0] * ub[0] + n[1] * ub[1] + n[2] * ub[2];
    const double a = un + phi / h;
    if (a > 0.0) {
        v[0] = ub[0]; v[1] = ub[1]; v[2] = ub[2];
        f[0] = f[1] = f[2] = 0.0;
        return TAKEOFF;
    }
    const double ut0 = ub[0] - un * n[0], ut1 = ub[1] - un * n[1], ut2 = ub[2] - un * n[2];
    const double tau = sqrt(ut0 * ut0 + ut1 * ut1 + ut2 * ut2);
    const double vn = -phi / h;
    uint8_t md;
    if (tau <= mu * (-a)) {
        v[0] = vn * n[0]; v[1] = vn * n[1]; v[2] = vn * n[2];
        md = STICK;
    } else {
        const double k = mu * a / tau;
        v[0] = vn * n[0] + ut0 + k * ut0;
        v[1] = vn * n[1] + ut1 + k * ut1;
        v[2] = vn * n[2] + ut2 + k * ut2;
        md = SLIP;
    }
    f[0] = mass * (v[0] - ub[0]);
    f[1] = mass * (v[1] - ub[1]);
    f[2] = mass * (v[2] - ub[2]);
    return md;
}

// ------------------------------------------------------------------ forward

// w_c p_c for active constraints [c0, c1) at x^k = x_n + h v^k (local step,
// constraint-centred; used for curved bending stencils).
template <bool MIXED>
__device__ __forceinline__ void local_projection(const SimDev &S, auto XN, auto vk, int c0, int c1) {
    const double h = S.h;
    for (int c = c0 + threadIdx.x; c < c1; c += (int)blockDim.x) {
        double q0 = 0, q1 = 0, q2 = 0;
        for (int p = G(S.c_ptr)[c]; p < G(S.c_ptr)[c + 1]; ++p) {
            const int j = G(S.c_node)[p];
            const double a = G(S.c_coef)[p];
            q0 += a * (XN[3 * j] + h * vk[3 * j]);
            q1 += a * (XN[3 * j + 1] + h * vk[3 * j + 1]);
            q2 += a * (XN[3 * j + 2] + h * vk[3 * j + 2]);
        }
        double p0, p1, p2;
        if (MIXED) {
            const float f0 = (float)q0, f1 = (float)q1, f2 = (float)q2;
            const float nq = sqrtf(f0 * f0 + f1 * f1 + f2 * f2);
            const float rho = G(S.c_rhof)[c], w = G(S.c_wf)[c];
            float r0, r1, r2;
            if (nq < 1e-12f * rho) {
                r0 = rho * (float)G(S.c_restdir)[3 * c]; r1 = rho * (float)G(S.c_restdir)[3 * c + 1];
                r2 = rho * (float)G(S.c_restdir)[3 * c + 2];
            } else {
                const float sc = rho / nq;
                r0 = sc * f0; r1 = sc * f1; r2 = sc * f2;
            }
            p0 = (double)(w * r0); p1 = (double)(w * r1); p2 = (double)(w * r2);
        } else {
            const double nq = sqrt(q0 * q0 + q1 * q1 + q2 * q2);
            const double rho = G(S.c_rho)[c], w = G(S.c_w)[c];
            if (nq < 1e-12 * rho) {
                p0 = w * rho * G(S.c_restdir)[3 * c]; p1 = w * rho * G(S.c_restdir)[3 * c + 1];
                p2 = w * rho * G(S.c_restdir)[3 * c + 2];
            } else {
                const double sc = w * rho / nq;
                p0 = sc * q0; p1 = sc * q1; p2 = sc * q2;
            }
        }
        G(S.wp)[3 * c] = p0; G(S.wp)[3 * c + 1] = p1; G(S.wp)[3 * c + 2] = p2;
    }
}

// Right-hand side of the global step (eqn pd_velocity_with_contact), nodes
// [i0, i1): out_i = b0_i + h sum_c a_ci w_c p_c + f_i.  Springs are projected here,
// node-centred (each spring on both of its nodes, with the same arithmetic, so
// the two contributions are exact negatives); curved-bending projections come
// from wp.
template <bool MIXED>
__device__ __forceinline__ void spring_rhs(const SimDev &S, auto XN, auto V, auto out, int i0, int i1) {
    const double h = S.h;
    const bool bend = S.nca_bend > 0;
    for (int i = i0 + (int)threadIdx.x; i < i1; i += (int)blockDim.x) {
        double r0 = 0, r1 = 0, r2 = 0;
        const int p0 = G(S.sinc_ptr)[i], p1 = G(S.sinc_ptr)[i + 1];
        // q = (x_i + h v_i) - (x_j + h v_j) = sign (x_a - x_b) exactly, so the
        // two nodes of a spring add exact negatives
        const double y0 = XN[3 * i] + h * V[3 * i], y1 = XN[3 * i + 1] + h * V[3 * i + 1],
                     y2 = XN[3 * i + 2] + h * V[3 * i + 2];
        const auto rec = (GLOBAL const v4i *)S.sinc;       // SpringInc as 16 bytes
        for (int pb = p0; pb < p1; pb += 8) {
            v4i spv[8];
            double rhov[8];
#pragma unroll
            for (int j = 0; j < 8; ++j)                      // independent record loads in flight
                if (pb + j < p1) { spv[j] = rec[pb + j]; rhov[j] = G(S.sinc_rho)[pb + j]; }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (pb + j >= p1) break;
                const int nj = spv[j].x, cs = spv[j].y;
                const double wr = __longlong_as_double(((long long)spv[j].w << 32) | (uint32_t)spv[j].z);
                const double q0 = y0 - (XN[3 * nj] + h * V[3 * nj]);
                const double q1 = y1 - (XN[3 * nj + 1] + h * V[3 * nj + 1]);
                const double q2 = y2 - (XN[3 * nj + 2] + h * V[3 * nj + 2]);
                double p0v, p1v, p2v;
                if (MIXED) {
                    const float f0 = (float)q0, f1 = (float)q1, f2 = (float)q2;
                    const float nq = sqrtf(f0 * f0 + f1 * f1 + f2 * f2);
                    const float wrf = (float)wr;
                    if (nq < 1e-12f * (float)rhov[j]) {
                        const auto rd = G(S.c_restdir) + 3 * (cs >= 0 ? cs : ~cs);
                        const float sg = cs >= 0 ? wrf : -wrf;
                        p0v = (double)(sg * (float)rd[0]); p1v = (double)(sg * (float)rd[1]); p2v = (double)(sg * (float)rd[2]);
                    } else {
                        const float sc = wrf / nq;
                        p0v = (double)(sc * f0); p1v = (double)(sc * f1); p2v = (double)(sc * f2);
                    }
                } else {
                    const double nq = sqrt(q0 * q0 + q1 * q1 + q2 * q2);
                    if (nq < 1e-12 * rhov[j]) {
                        const auto rd = G(S.c_restdir) + 3 * (cs >= 0 ? cs : ~cs);
                        const double sg = cs >= 0 ? wr : -wr;
                        p0v = sg * rd[0]; p1v = sg * rd[1]; p2v = sg * rd[2];
                    } else {
                        const double sc = wr / nq;
                        p0v = sc * q0; p1v = sc * q1; p2v = sc * q2;
                    }
                }
                r0 += p0v; r1 += p1v; r2 += p2v;
            }
        }
        if (bend) {
            for (int p = G(S.binc_ptr)[i]; p < G(S.binc_ptr)[i + 1]; ++p) {
                const int c = G(S.binc_con)[p];
                const double a = G(S.binc_coef)[p];
                r0 += a * G(S.wp)[3 * c]; r1 += a * G(S.wp)[3 * c + 1]; r2 += a * G(S.wp)[3 * c + 2];
            }
        }
        out[3 * i] = G(S.b0)[3 * i] + h * r0 + G(S.f)[3 * i];
        out[3 * i + 1] = G(S.b0)[3 * i + 1] + h * r1 + G(S.f)[3 * i + 1];
        out[3 * i + 2] = G(S.b0)[3 * i + 2] + h * r2 + G(S.f)[3 * i + 2];
    }
}


// Forward prefetch workgroup j of H (same XCD as the solving workgroup of
// its handle): follows the announced solve phases and touches every 128-byte
// line of the blocks of the next phase; returns when the solver is done or
// nothing new was announced for 100 ms.
__device__ void fwd_prefetch(const SimDev &S, int j, int H) {
    __shared__ int go;
    const int PH = 2 * S.n_levels;
    const int64_t stride = (int64_t)H * blockDim.x, me = (int64_t)j * blockDim.x + threadIdx.x;
    uint64_t sink = 0;
    for (int64_t target = 0;; ++target) {
        if (threadIdx.x == 0) {
            int state = 0;                                   // 0: give up, 1: go, 2: solver done
            const uint64_t t0 = wall_clock64();
            while (wall_clock64() - t0 < 10000000ull) {      // 100 ms at the 100 MHz wall clock
                const int64_t p = __hip_atomic_load(S.fwd_pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((p >> 40) == S.fwd_epoch) {
                    const int64_t pm = p & kPosMask;
                    if (pm == kPosMask) { state = 2; break; }
                    if (pm + 1 >= target) { state = 1; break; }
                }
                __builtin_amdgcn_s_sleep(2);
            }
            go = state;
        }
        __syncthreads();
        const int st = go;
        __syncthreads();
        if (st != 1) break;
        const int q = (int)(target % PH);
        const auto base = G(q < S.n_levels ? S.gval : S.gvalt);
        int64_t line0 = 0;
        for (int r = G(S.fpf_ptr)[q]; r < G(S.fpf_ptr)[q + 1]; ++r) {
            const int64_t o = G(S.fpf)[2 * r], len = G(S.fpf)[2 * r + 1];
            const int64_t nl = (len + 15) / 16;
            int64_t i = (me - line0) % stride;
            if (i < 0) i += stride;
            for (; i < nl; i += stride) {
                sink ^= (uint64_t)__double_as_longlong(base[o + 16 * i]);
                if (i == nl - 1) sink ^= (uint64_t)__double_as_longlong(base[o + len - 1]);
            }
            line0 += nl;
        }
    }
    if (sink == 0x9e3779b97f4a7c15ull) G(S.red)[62] = 1.0;         // keeps the loads
}

// Step prologue of node i: predictor, detection on y, constant right-hand
// side, initial guess and impulses; the external force f_ext = M g + fs F
// enters all four.  KX: also copy x_n to XN (positions placed in LDS).
template <bool km, bool KX>
__device__ __forceinline__ void fwd_prologue_node(const SimDev &S, int i, double fs, double t1, bool first,
                                                  GLOBAL double *xrec, GLOBAL double *vrec, auto A, auto XN) {
    const double h = S.h;
    const double xi[3] = {G(S.x)[3 * i], G(S.x)[3 * i + 1], G(S.x)[3 * i + 2]};
    const double vi[3] = {G(S.v)[3 * i], G(S.v)[3 * i + 1], G(S.v)[3 * i + 2]};
    if (first) {
        for (int d = 0; d < 3; ++d) { xrec[3 * i + d] = xi[d]; vrec[3 * i + d] = vi[d]; }
    }
    const double mi = G(S.mass)[i];
    double fe[3] = {0.0, 0.0, 0.0}, ae[3];           // external force, M^{-1} f_ext
    if (S.fext != nullptr)
        for (int d = 0; d < 3; ++d) fe[d] = fs * G(S.fext)[3 * i + d];
    for (int d = 0; d < 3; ++d) ae[d] = S.g[d] + fe[d] / mi;
    double y[3];
    {
#pragma clang fp contract(off)                       // (x + h v) + (h h) a, unfused: see mesh_frame
        for (int d = 0; d < 3; ++d) y[d] = xi[d] + h * vi[d] + h * h * ae[d];
    }
    double best = 0.0;
    int ob = -1;
    for (int o = 0; o < S.n_obst; ++o) {
        const double phi = signed_distance<km>(S.obst[o], y);
        if (ob < 0 || phi < best) { best = phi; ob = o; }
    }
    const bool contact = ob >= 0 && best <= 0.0;
    G(S.mode)[i] = contact ? TAKEOFF : FREE;
    G(S.cobst)[i] = contact ? (int8_t)ob : (int8_t)-1;
    if constexpr (km) {
        if (contact && S.obst[ob].type == 2) {     // the step's frame at x_n, scanned once
            double nr[3], ph;
            contact_frame<true>(S, ob, xi, nr, ph);
            for (int d = 0; d < 3; ++d) G(S.cfr)[8 * i + d] = nr[d];
            G(S.cfr)[8 * i + 3] = ph;
        }
    }
    double kx0 = 0, kx1 = 0, kx2 = 0;
    for (int p = G(S.ks_ptr)[i]; p < G(S.ks_ptr)[i + 1]; ++p) {
        const int j = G(S.ks_col)[p];
        const double kv = G(S.ks_val)[p];
        kx0 += kv * G(S.x)[3 * j];
        kx1 += kv * G(S.x)[3 * j + 1];
        kx2 += kv * G(S.x)[3 * j + 2];
    }
    double b[3] = {mi * vi[0] + h * (mi * S.g[0] + fe[0]) - h * kx0,
                   mi * vi[1] + h * (mi * S.g[1] + fe[1]) - h * kx1,
                   mi * vi[2] + h * (mi * S.g[2] + fe[2]) - h * kx2};
    const int as = G(S.att_of)[i];
    if (as >= 0) {
        double tg[3];
        attach_target(S, G(S.att_rest) + 3 * as, t1, tg);
        for (int d = 0; d < 3; ++d) b[d] += h * S.w_att * tg[d];
    }
    if (S.self_on)
        for (int d = 0; d < 3; ++d) G(S.ybuf)[3 * i + d] = y[d];
    // impulses: zero, or (warm start) the previous step's on the nodes of
    // this step's contact set (zero where the node was not in contact; with
    // self-collision every node keeps its impulse until the pairs are known)
    const bool keep = S.warm_start && (contact || S.self_on);
    for (int d = 0; d < 3; ++d) {
        G(S.b0)[3 * i + d] = b[d];
        if (!keep) G(S.f)[3 * i + d] = 0.0;
        A[3 * i + d] = vi[d] + h * ae[d];
    }
    if constexpr (KX)
        for (int d = 0; d < 3; ++d) XN[3 * i + d] = xi[d];
}

// ------------------------------------------------------------------ node-node self-collision

// Nodes i and j share a constraint stencil (never a pair).
__device__ __forceinline__ bool self_adjacent(const SimDev &S, int i, int j) {
    for (int p = G(S.adj_ptr)[i]; p < G(S.adj_ptr)[i + 1]; ++p)
        if (G(S.adj_col)[p] == j) return true;
    return false;
}

// Uniform grid over the predictor with cells no smaller than the detection
// radius, hashed into a table of linked lists (the spatial hashing of
// Teschner et al., "Optimized Spatial Hashing for Collision Detection of
// Deformable Objects", VMV 2003): every node within the radius of y_i lies in
// one of the 27 cells around y_i's cell.  Bucket lists are built with atomic
// exchanges, so their order varies from run to run; the search below takes a
// minimum under a total order, so its result does not.
__device__ __forceinline__ int self_cell(double y, double inv) {
    return (int)floor(fmin(fmax(y * inv, -1.0e9), 1.0e9));
}
__device__ __forceinline__ int self_bucket(const SimDev &S, int cx, int cy, int cz) {
    return (int)(((uint32_t)cx * 73856093u ^ (uint32_t)cy * 19349663u ^ (uint32_t)cz * 83492791u) &
                 (uint32_t)S.self_hmask);
}
__device__ __forceinline__ int32_t self_load(GLOBAL int32_t *p) {   // past any stale cached copy
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void self_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Node i (outside the obstacle contact set) joins the bucket of its cell.
__device__ __forceinline__ void self_insert(const SimDev &S, int i) {
    if (G(S.mode)[i] != FREE) return;
    const double inv = S.self_inv_cell;
    const int b = self_bucket(S, self_cell(G(S.ybuf)[3 * i], inv), self_cell(G(S.ybuf)[3 * i + 1], inv),
                              self_cell(G(S.ybuf)[3 * i + 2], inv));
    G(S.self_next)[i] = __hip_atomic_exchange(G(S.self_head) + b, i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Nearest eligible node of node i on the predictor (Sec. 4.2, Extensions):
// both nodes outside the obstacle contact set, not sharing a stencil, apart at
// x_n, |y_i - y_j|^2 <= r^2 (squared distances summed over x, y, z in that
// order, unfused); ties to the lower caller id.  Candidates come from the 27
// grid cells around y_i (a bucket met twice is scanned twice, harmlessly).
__device__ __forceinline__ void self_nearest(const SimDev &S, int i, auto XN) {
#pragma clang fp contract(off)
    int best = -1;
    double bd = 0.0;
    if (G(S.mode)[i] == FREE) {
        const double y0 = G(S.ybuf)[3 * i], y1 = G(S.ybuf)[3 * i + 1], y2 = G(S.ybuf)[3 * i + 2];
        const double inv = S.self_inv_cell;
        const int cx = self_cell(y0, inv), cy = self_cell(y1, inv), cz = self_cell(y2, inv);
        for (int q = 0; q < 27; ++q) {
            const int b = self_bucket(S, cx + q % 3 - 1, cy + (q / 3) % 3 - 1, cz + q / 9 - 1);
            for (int j = self_load(G(S.self_head) + b); j >= 0; j = self_load(G(S.self_next) + j)) {
                const double e0 = y0 - G(S.ybuf)[3 * j], e1 = y1 - G(S.ybuf)[3 * j + 1], e2 = y2 - G(S.ybuf)[3 * j + 2];
                const double d2 = e0 * e0 + e1 * e1 + e2 * e2;
                if (!(d2 <= S.self_r2) || j == i) continue;
                if (best >= 0 && (d2 > bd || (d2 == bd && G(S.caller_id)[j] >= G(S.caller_id)[best]))) continue;
                const double x0 = XN[3 * i] - XN[3 * j], x1 = XN[3 * i + 1] - XN[3 * j + 1],
                             x2 = XN[3 * i + 2] - XN[3 * j + 2];
                if (!(x0 * x0 + x1 * x1 + x2 * x2 > 0.0) || self_adjacent(S, i, j)) continue;
                best = j;
                bd = d2;
            }
        }
    }
    G(S.cand)[i] = best;
}

// Pairs are the mutually nearest nodes; a pair node enters the contact set.
// Impulses: a pair starts from zero or (warm start) from its leader's impulse
// at the end of the previous step (the follower takes its negative); nodes in
// no contact start from zero.
__device__ __forceinline__ void self_pair_setup(const SimDev &S, int i) {
    const int c = G(S.cand)[i];
    const int p = (c >= 0 && G(S.cand)[c] == i) ? c : -1;
    G(S.partner)[i] = p;
    if (p >= 0) {
        G(S.mode)[i] = TAKEOFF;
        if (G(S.caller_id)[i] > G(S.caller_id)[p])            // follower (the leader keeps its own)
            for (int d = 0; d < 3; ++d) G(S.f)[3 * i + d] = S.warm_start ? -G(S.f)[3 * p + d] : 0.0;
    } else if (G(S.mode)[i] == FREE) {
        for (int d = 0; d < 3; ++d) G(S.f)[3 * i + d] = 0.0;
    }
}

// Pair frame at x_n: n = (x_L - x_F) / r, gap r - d (L the leader).
__device__ __forceinline__ void self_frame(const SimDev &S, int L, int F, auto XN, double *n, double &phi,
                                           double &r) {
    const double e0 = XN[3 * L] - XN[3 * F], e1 = XN[3 * L + 1] - XN[3 * F + 1], e2 = XN[3 * L + 2] - XN[3 * F + 2];
    r = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
    n[0] = e0 / r; n[1] = e1 / r; n[2] = e2 / r;
    phi = r - S.self_d;
}

// Contact update of a pair, run by its leader L for both nodes: the free
// velocities ub_L = v_L - f/m_L, ub_F = v_F + f/m_F, the closed-form law on
// their difference with the reduced mass, then v_L = ub_L + f'/m_L,
// v_F = ub_F - f'/m_F; both nodes' share of the iteration's change.
__device__ __forceinline__ void self_pair_update(const SimDev &S, int L, int F, auto B, auto XN, auto Vprev,
                                                 bool converge, double &dmax) {
    const double mL = G(S.mass)[L], mF = G(S.mass)[F];
    double ubL[3], ubF[3], ur[3], fp[3];
    for (int d = 0; d < 3; ++d) {
        fp[d] = G(S.f)[3 * L + d];
        ubL[d] = B[3 * L + d] - fp[d] / mL;
        ubF[d] = B[3 * F + d] + fp[d] / mF;
        ur[d] = ubL[d] - ubF[d];
    }
    double nrm[3], phi, r, u[3], fn[3];
    self_frame(S, L, F, XN, nrm, phi, r);
    const double mred = mL * mF / (mL + mF);
    const uint8_t md = signorini_coulomb(ur, nrm, phi, S.self_mu, S.h, mred, u, fn);
    G(S.mode)[L] = md;
    G(S.mode)[F] = md;
    for (int d = 0; d < 3; ++d) {
        const double vL = ubL[d] + fn[d] / mL, vF = ubF[d] - fn[d] / mF;
        if (converge) {
            dmax = fmax(dmax, fmax(fabs(fn[d] - fp[d]) / mL, fabs(fn[d] - fp[d]) / mF));
            dmax = fmax(dmax, fmax(fabs(vL - Vprev[3 * L + d]), fabs(vF - Vprev[3 * F + d])));
        }
        B[3 * L + d] = vL;
        B[3 * F + d] = vF;
        G(S.f)[3 * L + d] = fn[d];
        G(S.f)[3 * F + d] = -fn[d];
        G(S.ubar)[3 * L + d] = ubL[d];
        G(S.ubar)[3 * F + d] = ubF[d];
    }
}

// Contact update of node i after a global solve (its new velocity in B), and
// the node's share of the iteration's change max(|dv|, |df| / m).  A pair
// node: its leader updates both nodes (the follower does nothing here).
template <bool km>
__device__ __forceinline__ void fwd_contact_node(const SimDev &S, int i, auto B, auto XN, auto Vprev, bool converge,
                                                 double &dmax) {
    const double h = S.h;
    if (S.self_on) {
        const int p = G(S.partner)[i];
        if (p >= 0) {
            if (G(S.caller_id)[i] < G(S.caller_id)[p]) self_pair_update(S, i, p, B, XN, Vprev, converge, dmax);
            return;
        }
    }
    if (G(S.mode)[i] != FREE) {
        const double mi = G(S.mass)[i];
        const double ub[3] = {B[3 * i] - G(S.f)[3 * i] / mi, B[3 * i + 1] - G(S.f)[3 * i + 1] / mi,
                              B[3 * i + 2] - G(S.f)[3 * i + 2] / mi};
        double nrm[3], phi, vv[3], ff[3];
        bool cached = false;                            // mesh: the frame of the step's start
        if constexpr (km) cached = S.obst[G(S.cobst)[i]].type == 2;
        if (cached) {
            for (int d = 0; d < 3; ++d) nrm[d] = G(S.cfr)[8 * i + d];
            phi = G(S.cfr)[8 * i + 3];
        } else {
            contact_frame<false>(S, G(S.cobst)[i], XN + 3 * i, nrm, phi);
        }
        G(S.mode)[i] = signorini_coulomb(ub, nrm, phi, S.obst[G(S.cobst)[i]].mu, h, mi, vv, ff);
        for (int d = 0; d < 3; ++d) {
            // the iterate is (v, f): a node held by the contact update
            // keeps its velocity while its impulse may still change
            if (converge) dmax = fmax(dmax, fabs(ff[d] - G(S.f)[3 * i + d]) / mi);
            B[3 * i + d] = vv[d];
            G(S.f)[3 * i + d] = ff[d];
            G(S.ubar)[3 * i + d] = ub[d];
        }
    }
    if (converge)
        for (int d = 0; d < 3; ++d) dmax = fmax(dmax, fabs(B[3 * i + d] - Vprev[3 * i + d]));
}

// Advance and record node i (the converged iterate is in A); counts its mode.
__device__ __forceinline__ void fwd_record_node(const SimDev &S, int i, int slot, auto A, auto XN, GLOBAL double *xn,
                                                GLOBAL double *vn, GLOBAL double *ubrec, int *cnt) {
    const int m = S.m;
    const double h = S.h;
    for (int d = 0; d < 3; ++d) {
        const double vv = A[3 * i + d];
        const double xx = XN[3 * i + d] + h * vv;
        G(S.x)[3 * i + d] = xx;
        G(S.v)[3 * i + d] = vv;
        xn[3 * i + d] = xx;
        vn[3 * i + d] = vv;
        ubrec[3 * i + d] = G(S.ubar)[3 * i + d];
    }
    const uint8_t md = G(S.mode)[i];
    if (md != FREE) ++cnt[md - 1];
    G(S.rec_mode)[(int64_t)slot * m + i] = md;
    G(S.rec_obst)[(int64_t)slot * m + i] = G(S.cobst)[i];
    if (S.self_on) G(S.rec_partner)[(int64_t)slot * m + i] = G(S.partner)[i];
}

// per-step record of step n: PD iterations and mode counts
__device__ __forceinline__ void put_step_info(const SimDev &S, int n, int k, int64_t takeoff, int64_t stick,
                                              int64_t slip) {
    if (S.step_info != nullptr) {
        G(S.step_info)[4 * n] = k;
        G(S.step_info)[4 * n + 1] = (int32_t)takeoff;
        G(S.step_info)[4 * n + 2] = (int32_t)stick;
        G(S.step_info)[4 * n + 3] = (int32_t)slip;
    }
}

// Forward steps [step_begin, step_end) of one handle per workgroup.  The PD
// iterate ping-pongs between two vectors A and B (LDS when they fit): B gets
// the right-hand side, the forward solve writes into A, the backward solve
// writes the new iterate into B.  With helpers > 0 the launch also holds
// prefetch workgroups (see fwd_prefetch) laid out by XCD.
template <bool MIXED, int FL>
__global__ __launch_bounds__(kBlock) void k_forward(const SimDev *__restrict__ sims, int nsims, int helpers) {
    int hid = blockIdx.x;
    if (helpers > 0) {          // workgroup 8 j + x: handle (j / (H+1)) 8 + x, role j mod (H+1) (0: solver)
        const int x = (int)blockIdx.x % kXcds, jj = (int)blockIdx.x / kXcds;
        hid = jj / (helpers + 1) * kXcds + x;
        const int role = jj % (helpers + 1);
        if (hid >= nsims) return;
        if (role > 0) {
            fwd_prefetch(sims[hid], role - 1, helpers);
            return;
        }
    }
    const SimDev &S = sims[hid];
    extern __shared__ double dyn[];
    __shared__ double red[kBlock / 64];
    const int m = S.m;
    const double h = S.h;
    const bool converge = S.fwd_tol > 0;
    constexpr bool kv = (FL & kLdsVectors) != 0, ku = (FL & kLdsUpdates) != 0, kx = (FL & kLdsPositions) != 0;
    constexpr bool km = (FL & kMeshObst) != 0;
    const int off_u = kv ? 6 * m : 0, off_x = off_u + (ku ? S.n_ubuf : 0);
    auto A = pick<kv>(dyn, G(S.vk));
    auto B = pick<kv>(dyn + 3 * m, G(S.rhs));
    auto U = pick<ku>(dyn + off_u, G(S.ubuf));
    auto XN = pick<kx>(dyn + off_x, G(S.x));
    auto Vprev = G(S.vk1);
    int64_t iters_total = 0, it_run = 0;
    for (int n = S.step_begin; n < S.step_end; ++n) {
        const int slot = S.rec_ring ? 0 : n - S.rec_step0;
        const double t1 = (n + 1) * h;
        auto xrec = G(S.rec_x) + (int64_t)slot * 3 * m;
        auto vrec = G(S.rec_v) + (int64_t)slot * 3 * m;
        const double fs = S.fext == nullptr ? 0.0 : (S.fscale == nullptr ? 1.0 : G(S.fscale)[n]);
        for (int i = threadIdx.x; i < m; i += (int)blockDim.x)
            fwd_prologue_node<km, kx>(S, i, fs, t1, n == S.step_begin, xrec, vrec, A, XN);
        __syncthreads();
        if (S.self_on) {                                 // node-node contacts of this step
            // the grid's table is cleared and filled with atomics at the device's
            // L2: agent-scope fences around the barriers order plain stores,
            // atomics and loads of the lists
            for (int b = threadIdx.x; b <= S.self_hmask; b += (int)blockDim.x) G(S.self_head)[b] = -1;
            self_sync();
            for (int i = threadIdx.x; i < m; i += (int)blockDim.x) self_insert(S, i);
            self_sync();
            for (int i = threadIdx.x; i < m; i += (int)blockDim.x) self_nearest(S, i, XN);
            __syncthreads();
            for (int i = threadIdx.x; i < m; i += (int)blockDim.x) self_pair_setup(S, i);
            __syncthreads();
        }
        int k = 0;
        while (true) {
            if (S.nca_bend > 0) {
                local_projection<MIXED>(S, XN, A, S.nca - S.nca_bend, S.nca);
                __syncthreads();
            }
            spring_rhs<MIXED>(S, XN, A, B, 0, m);
            if (converge)
                for (int i = threadIdx.x; i < 3 * m; i += (int)blockDim.x) Vprev[i] = A[i];
            __syncthreads();
            solve_P(S, G(S.lvl_team), B, B, A, B, U, it_run * 2 * S.n_levels);
            ++it_run;
            double dmax = 0.0;
            for (int i = threadIdx.x; i < m; i += (int)blockDim.x) fwd_contact_node<km>(S, i, B, XN, Vprev, converge, dmax);
            ++k;
            auto tmp = A; A = B; B = tmp;
            if (converge) {
                dmax = block_max(dmax, red);          // includes the barrier
                if (!(dmax > S.fwd_tol) || k >= S.fwd_max_iters) break;
            } else {
                __syncthreads();
                if (k >= S.K) break;
            }
        }
        iters_total += k;
        // advance and record (the iterate is in A)
        auto xn = xrec + 3 * m;
        auto vn = vrec + 3 * m;
        auto ubrec = G(S.rec_ubar) + (int64_t)slot * 3 * m;
        int cnt[3] = {0, 0, 0};                          // take-off, stick, slip nodes of this thread
        for (int i = threadIdx.x; i < m; i += (int)blockDim.x) fwd_record_node(S, i, slot, A, XN, xn, vn, ubrec, cnt);
        // per-step record: iterations and mode counts (sums of small integers, exact in float64)
        const double packed = (double)cnt[0] + 1048576.0 * (double)cnt[1];   // counts < 2^20 per handle
        const double tot01 = block_sum(packed, red);
        const double tot2 = block_sum((double)cnt[2], red);
        if (threadIdx.x == 0) {
            const int64_t t01 = (int64_t)tot01;
            put_step_info(S, n, k, t01 & 1048575, t01 >> 20, (int64_t)tot2);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) G(S.counters)[0] += iters_total;
    announce(S.fwd_pos, S.fwd_epoch, kPosMask);          // releases the prefetch workgroups
}

// ------------------------------------------------------------------ multi-workgroup forward

// A right-hand-side vector held from column c0 on (the root's gathered rows in
// LDS), indexed with the global offsets the work items carry.
struct Shifted {
    double *p;
    int off;
    __device__ double &operator[](int i) const { return p[i - off]; }
    __device__ Shifted operator+(int k) const { return Shifted{p, off - k}; }
};

// Pairs of factor entries copied into LDS, indexed like the pairs in gval
// (pair index minus the copy's first pair), for fwd_products.
struct LdsPairs {
    const double *p;
    int off;
    __device__ LdsPairs operator+(int k) const { return LdsPairs{p, off - k}; }
    __device__ v2d operator[](int i) const {
        const int j = 2 * (i - off);
        return v2d{p[j], p[j + 1]};
    }
};

// Copies n doubles (n even, src 16-byte aligned) from global memory into LDS,
// the whole workgroup, four 16-byte loads per thread in flight.
__device__ __forceinline__ void lds_copy(double *dst, GLOBAL const double *src, int n) {
    const auto s2 = (GLOBAL const v2d *)src;
    const int np = n >> 1, bd = (int)blockDim.x;
    for (int j = (int)threadIdx.x; j < np; j += 4 * bd) {
        v2d v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = j + u * bd < np ? s2[j + u * bd] : v2d{0.0, 0.0};
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (j + u * bd < np) {
                dst[2 * (j + u * bd)] = v[u].x;
                dst[2 * (j + u * bd) + 1] = v[u].y;
            }
    }
}

// Barrier of the S.mw workgroups of a multi-workgroup forward launch (placed
// on one XCD).  An agent-scope release before arriving and an acquire after
// leaving make every workgroup's global writes visible to the others.  Thread
// 0 waits at most S.mw_spin ticks of the 100 MHz wall clock; then, or when
// another workgroup has already given up, it raises the failure flag, and
// every thread of the workgroup gets false (the kernel then returns and the
// host reports the failure).  gen: thread 0's count of barriers passed.
__device__ __forceinline__ bool mw_barrier(const SimDev &S, uint32_t &gen, int &ok_lds) {
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t *cnt = S.mw_sync, *gn = S.mw_sync + 1, *fail = S.mw_sync + 2;
        int ok = 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (__hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            ok = 0;
        } else {
            const uint32_t g = gen;
            const uint32_t arrived = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
            if (arrived == (uint32_t)S.mw) {
                __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(gn, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                const uint64_t t0 = wall_clock64();
                while (__hip_atomic_load(gn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                    if (__hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                        wall_clock64() - t0 > (uint64_t)S.mw_spin) {
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            gen = g + 1u;
        }
        if (!ok) __hip_atomic_store(fail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        ok_lds = ok;
    }
    __syncthreads();
    return ok_lds != 0;
}

// Forward steps [step_begin, step_end) of one handle on S.mw workgroups of one
// XCD (workgroups 8 w; the others of the grid return at once).  Workgroup w
// owns whole subtrees of the elimination tree below the root supernode and a
// slice of the root's columns (node ranges S.mw_nodes): it does their step
// prologue, right-hand side, both triangular solves and contact updates; the
// root's forward product (its stored inverse) is split over all workgroups in
// contiguous runs of row pairs, each of which first gathers the root's whole
// right-hand side into LDS; its run of the stored inverse is copied into LDS
// once per launch when it fits (S.mw_root_lds).
// Barriers per PD iteration: after the subtrees' forward solves, after the
// root product, after the contact updates (and after the bending projections
// when there are curved bending constraints).  Every node, row and item is
// computed with the arithmetic of k_forward (same items, team sizes and
// summation orders), so results are bitwise those of the single-workgroup
// kernel.  Vectors live in HBM and are shared through the XCD's L2.
template <bool MIXED, bool km, bool LW>
__global__ __launch_bounds__(kBlock) void k_forward_mw(const SimDev *__restrict__ sims) {
    if ((int)blockIdx.x % kXcds != 0) return;
    const SimDev &S = sims[0];
    const int W = S.mw, w = (int)blockIdx.x / kXcds;
    if (w >= W || (S.mw_absent && w == W - 1)) return;
    extern __shared__ double dyn[];
    __shared__ double red[kBlock / 64];
    __shared__ double troot[3 * kMwRootMax];
    __shared__ int ok_lds;
    uint32_t gen = 0;
    const int m = S.m, L = S.n_levels, Q = W * (L - 1);
    const double h = S.h;
    const bool converge = S.fwd_tol > 0;
    auto A = G(S.vk);
    auto B = G(S.rhs);
    auto U = G(S.ubuf);
    auto XN = G(S.x);
    auto Y = G(S.ysol);
    auto Vprev = G(S.vk1);
    const auto gv2 = (GLOBAL const v2d *)S.gval;
    const auto gt2 = (GLOBAL const v2d *)S.gvalt;
    auto part = (GLOBAL double *)(S.mw_sync + 4);         // partials: W maxima, then 2 W packed counts
    if (threadIdx.x == 0) gen = __hip_atomic_load(S.mw_sync + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ra[kMwRanges], rb[kMwRanges];
    for (int r = 0; r < kMwRanges; ++r) {
        ra[r] = G(S.mw_nodes)[2 * (w * kMwRanges + r)];
        rb[r] = G(S.mw_nodes)[2 * (w * kMwRanges + r) + 1];
    }
    auto own = [&](auto &&f) {
        for (int r = 0; r < kMwRanges; ++r)
            for (int i = ra[r] + (int)threadIdx.x; i < rb[r]; i += (int)blockDim.x) f(i);
    };
    const int rs0 = S.mw_root_c0, rn = S.n_root_rows;
    const int ys0 = rs0 + (int)((int64_t)rn * w / W), ys1 = rs0 + (int)((int64_t)rn * (w + 1) / W);
    // LW: the workgroup's one subtree (columns [lo, hi), update slots [ulo, uhi))
    // is solved in LDS: right-hand side / solution, forward result and update
    // buffer; what other workgroups read goes out to HBM (the root rows' update
    // entries after the forward solve, the new iterate after the contact update)
    const int lo = LW ? G(S.mw_win)[4 * w] : 0, hi = LW ? G(S.mw_win)[4 * w + 1] : 0;
    const int ulo = LW ? G(S.mw_win)[4 * w + 2] : 0, uhi = LW ? G(S.mw_win)[4 * w + 3] : 0;
    const int nl = hi - lo;
    const Shifted sB{dyn, 3 * lo}, sY{dyn + 3 * nl, 3 * lo}, sU{dyn + 6 * nl, ulo};
    auto TY = pick<LW>(sY, Y);                             // own rows of the solve's vectors
    auto TU = pick<LW>(sU, U);
    const int ria = G(S.mw_rootw)[4 * w], rib = G(S.mw_rootw)[4 * w + 1];
    const int rgb = G(S.mw_rootw)[4 * w + 2], rgc = G(S.mw_rootw)[4 * w + 3];
    double *rootG = dyn + S.mw_root_off;
    if (S.mw_root_lds) {                                   // this workgroup's run of the root's inverse
        lds_copy(rootG, G(S.gval) + rgb, rgc);
        __syncthreads();
    }
    int64_t iters_total = 0;
    for (int n = S.step_begin; n < S.step_end; ++n) {
        const int slot = S.rec_ring ? 0 : n - S.rec_step0;
        const double t1 = (n + 1) * h;
        auto xrec = G(S.rec_x) + (int64_t)slot * 3 * m;
        auto vrec = G(S.rec_v) + (int64_t)slot * 3 * m;
        const double fs = S.fext == nullptr ? 0.0 : (S.fscale == nullptr ? 1.0 : G(S.fscale)[n]);
        own([&](int i) { fwd_prologue_node<km, false>(S, i, fs, t1, n == S.step_begin, xrec, vrec, A, XN); });
        if (!mw_barrier(S, gen, ok_lds)) return;
        if (S.self_on) {            // node-node contacts: the grid, the search and the pairs over all workgroups
            const int hs = S.self_hmask + 1;
            for (int b = hs * w / W + (int)threadIdx.x; b < hs * (w + 1) / W; b += (int)blockDim.x)
                G(S.self_head)[b] = -1;
            if (!mw_barrier(S, gen, ok_lds)) return;
            own([&](int i) { self_insert(S, i); });
            if (!mw_barrier(S, gen, ok_lds)) return;
            own([&](int i) { self_nearest(S, i, XN); });
            if (!mw_barrier(S, gen, ok_lds)) return;
            own([&](int i) { self_pair_setup(S, i); });
            if (!mw_barrier(S, gen, ok_lds)) return;
        }
        int k = 0;
        while (true) {
            // the solve runs in place in B (or its LDS window), which changes
            // with every swap of the iterates
            auto TB = pick<LW>(sB, B);
            if (S.nca_bend > 0) {                          // curved bending: constraints split by workgroup
                const int c0 = S.nca - S.nca_bend, nb = S.nca_bend;
                local_projection<MIXED>(S, XN, A, c0 + (int)((int64_t)nb * w / W), c0 + (int)((int64_t)nb * (w + 1) / W));
                if (!mw_barrier(S, gen, ok_lds)) return;
            }
            if constexpr (LW) {
                spring_rhs<MIXED>(S, XN, A, sB, lo, hi);
                spring_rhs<MIXED>(S, XN, A, B, ys0, ys1);
            } else {
                for (int r = 0; r < kMwRanges; ++r)
                    if (rb[r] > ra[r]) spring_rhs<MIXED>(S, XN, A, B, ra[r], rb[r]);
            }
            if (converge) own([&](int i) { for (int d = 0; d < 3; ++d) Vprev[3 * i + d] = A[3 * i + d]; });
            __syncthreads();
            // forward solve of this workgroup's subtrees, level by level
            for (int l = 0; l < L - 1; ++l) {
                const int q = w * (L - 1) + l;
                const int tl = G(S.lvl_team)[2 * l];
                const int team = threadIdx.x / tl, lane = threadIdx.x % tl, nteams = (int)blockDim.x / tl;
                const int i0 = G(S.mw_ptr)[(Q + 1) + q], i1 = G(S.mw_ptr)[(Q + 1) + q + 1];
                const auto fit = (GLOBAL const v4i *)S.mw_fitems;
                v4i cur = {0, 0, 0, 0}, cur2 = {0, 0, 0, 0};
                if (i0 + team < i1) { cur = fit[2 * (i0 + team)]; cur2 = fit[2 * (i0 + team) + 1]; }
                gather_rows(G(S.mw_rows), G(S.upd_off), G(S.mw_ptr)[q], G(S.mw_ptr)[q + 1], TB, TB, TU);
                __syncthreads();
                fwd_products(fit, gv2, i0 + team, i1, nteams, tl, lane, cur, cur2, TB, TY, TU);
                __syncthreads();
            }
            if constexpr (LW) {                            // the root rows' update entries, for every workgroup
                const auto bg = (GLOBAL const v2i *)S.mw_bgat;
                const int g0 = G(S.mw_ptr)[3 * (Q + 1) + w * (L - 1)], g1 = G(S.mw_ptr)[3 * (Q + 1) + (w + 1) * (L - 1)];
                for (int q = g0 + (int)threadIdx.x; q < g1; q += (int)blockDim.x) {
                    const v2i e = bg[q];
                    if (e.y < 0) { U[e.x] = sU[e.x]; U[e.x + 1] = sU[e.x + 1]; U[e.x + 2] = sU[e.x + 2]; }
                }
            }
            if (!mw_barrier(S, gen, ok_lds)) return;       // every subtree's updates of the root rows are in U
            {   // the root: its right-hand side gathered here, this workgroup's run of its product
                const int l = L - 1;
                const int tl = G(S.lvl_team)[2 * l];
                const int team = threadIdx.x / tl, lane = threadIdx.x % tl, nteams = (int)blockDim.x / tl;
                const auto fit = (GLOBAL const v4i *)S.fitems;
                const int t0 = ria + team;
                v4i cur = {0, 0, 0, 0}, cur2 = {0, 0, 0, 0};
                if (t0 < rib) { cur = fit[2 * t0]; cur2 = fit[2 * t0 + 1]; }
                const Shifted T{troot, 3 * rs0};
                gather_rows(G(S.rows), G(S.upd_off), G(S.lvl_rows_ptr)[l], G(S.lvl_rows_ptr)[l + 1], B, T, U);
                __syncthreads();
                if (S.mw_root_lds)
                    fwd_products(fit, LdsPairs{rootG, rgb >> 1}, t0, rib, nteams, tl, lane, cur, cur2, T, Y, U);
                else
                    fwd_products(fit, gv2, t0, rib, nteams, tl, lane, cur, cur2, T, Y, U);
            }
            if (!mw_barrier(S, gen, ok_lds)) return;       // the root's x (in Y) is complete
            // backward solve of this workgroup's subtrees, top level first
            for (int l = L - 2; l >= 0; --l) {
                const int q = w * (L - 1) + l;
                const int tl = G(S.lvl_team)[2 * l + 1];
                const int team = threadIdx.x / tl, lane = threadIdx.x % tl, nteams = (int)blockDim.x / tl;
                const int c0 = G(S.mw_ptr)[2 * (Q + 1) + q], c1 = G(S.mw_ptr)[2 * (Q + 1) + q + 1];
                const int q0 = G(S.mw_ptr)[3 * (Q + 1) + q], q1 = G(S.mw_ptr)[3 * (Q + 1) + q + 1];
                const auto bit = (GLOBAL const v4i *)S.mw_bitems;
                v4i cur = {0, 0, 0, 0}, cur2 = {0, 0, 0, 0};
                if (c0 + team < c1) { cur = bit[2 * (c0 + team)]; cur2 = bit[2 * (c0 + team) + 1]; }
                if (q1 > q0) {
                    bwd_gather((GLOBAL const v2i *)S.mw_bgat, q0, q1, threadIdx.x, blockDim.x, TB, Y, TU);
                    __syncthreads();
                }
                bwd_products(bit, gt2, c0 + team, c1, nteams, tl, lane, cur, cur2, TY, TB, TU);
                __syncthreads();
            }
            for (int i = ys0 + (int)threadIdx.x; i < ys1; i += (int)blockDim.x)   // this slice of the root: x from Y
                for (int d = 0; d < 3; ++d) B[3 * i + d] = Y[3 * i + d];
            __syncthreads();
            if (S.self_on)              // a pair's leader reads its follower's new velocity, maybe another's
                if (!mw_barrier(S, gen, ok_lds)) return;
            double dmax = 0.0;
            if constexpr (LW) {
                for (int i = lo + (int)threadIdx.x; i < hi; i += (int)blockDim.x) {
                    fwd_contact_node<km>(S, i, sB, XN, Vprev, converge, dmax);
                    for (int d = 0; d < 3; ++d) B[3 * i + d] = sB[3 * i + d];     // the new iterate, for every workgroup
                }
                for (int i = ys0 + (int)threadIdx.x; i < ys1; i += (int)blockDim.x)
                    fwd_contact_node<km>(S, i, B, XN, Vprev, converge, dmax);
            } else {
                own([&](int i) { fwd_contact_node<km>(S, i, B, XN, Vprev, converge, dmax); });
            }
            ++k;
            auto tmp = A; A = B; B = tmp;
            if (converge) {
                dmax = block_max(dmax, red);
                if (threadIdx.x == 0) part[w] = dmax;
                if (!mw_barrier(S, gen, ok_lds)) return;
                double mx = 0.0;
                for (int q = 0; q < W; ++q) mx = fmax(mx, part[q]);
                if (!(mx > S.fwd_tol) || k >= S.fwd_max_iters) break;
            } else {
                if (!mw_barrier(S, gen, ok_lds)) return;
                if (k >= S.K) break;
            }
        }
        iters_total += k;
        auto xn = xrec + 3 * m;
        auto vn = vrec + 3 * m;
        auto ubrec = G(S.rec_ubar) + (int64_t)slot * 3 * m;
        int cnt[3] = {0, 0, 0};
        own([&](int i) { fwd_record_node(S, i, slot, A, XN, xn, vn, ubrec, cnt); });
        const double packed = (double)cnt[0] + 1048576.0 * (double)cnt[1];
        const double tot01 = block_sum(packed, red);
        const double tot2 = block_sum((double)cnt[2], red);
        if (threadIdx.x == 0) {
            part[W + 2 * w] = tot01;
            part[W + 2 * w + 1] = tot2;
        }
        if (!mw_barrier(S, gen, ok_lds)) return;           // also: x_{n+1} of every node before the next prologue
        if (w == 0 && threadIdx.x == 0) {
            int64_t a = 0, b = 0, c = 0;
            for (int q = 0; q < W; ++q) {
                const int64_t t01 = (int64_t)part[W + 2 * q];
                a += t01 & 1048575;
                b += t01 >> 20;
                c += (int64_t)part[W + 2 * q + 1];
            }
            put_step_info(S, n, k, a, b, c);
        }
    }
    if (w == 0 && threadIdx.x == 0) G(S.counters)[0] += iters_total;
}

// ------------------------------------------------------------------ adjoint

// z = T^T zeta per node (T = I off contact / take-off, 0 for stick, the slip
// block otherwise); also keeps zeta - z for the (P - M) term.  A pair (L, F) in
// stick or slip with relative block T_r (in tblk of both nodes) and
// D = T_r - I enters in the mass-weighted form M T M^{-1}:
// z_L = zeta_L + (m_LF/m_L) D^T (zeta_L - zeta_F),
// z_F = zeta_F - (m_LF/m_F) D^T (zeta_L - zeta_F)  (m_LF the reduced mass).
__device__ __forceinline__ void apply_TT(const SimDev &S, auto mode, auto prt, auto zeta, auto z) {
    for (int i = threadIdx.x; i < S.m; i += (int)blockDim.x) {
        const uint8_t md = mode[i];
        const double a0 = zeta[3 * i], a1 = zeta[3 * i + 1], a2 = zeta[3 * i + 2];
        const int p = S.self_on ? prt[i] : -1;
        if (md == FREE || md == TAKEOFF) {
            z[3 * i] = a0; z[3 * i + 1] = a1; z[3 * i + 2] = a2;
        } else if (p >= 0) {
            const bool lead = G(S.caller_id)[i] < G(S.caller_id)[p];
            const int L = lead ? i : p, F = lead ? p : i;
            const double mL = G(S.mass)[L], mF = G(S.mass)[F];
            const double sa = (lead ? 1.0 : -1.0) * (mL * mF / (mL + mF)) / G(S.mass)[i];
            const double e[3] = {zeta[3 * L] - zeta[3 * F], zeta[3 * L + 1] - zeta[3 * F + 1],
                                 zeta[3 * L + 2] - zeta[3 * F + 2]};
            double De[3];                                    // D^T e
            if (md == STICK) {
                De[0] = -e[0]; De[1] = -e[1]; De[2] = -e[2];
            } else {
                const auto T = G(S.tblk) + 9 * (int64_t)i;
                for (int c = 0; c < 3; ++c) De[c] = T[c] * e[0] + T[3 + c] * e[1] + T[6 + c] * e[2] - e[c];
            }
            z[3 * i] = a0 + sa * De[0]; z[3 * i + 1] = a1 + sa * De[1]; z[3 * i + 2] = a2 + sa * De[2];
        } else if (md == STICK) {
            z[3 * i] = 0.0; z[3 * i + 1] = 0.0; z[3 * i + 2] = 0.0;
        } else {
            const auto T = G(S.tblk) + 9 * (int64_t)i;       // row-major T
            z[3 * i] = T[0] * a0 + T[3] * a1 + T[6] * a2;
            z[3 * i + 1] = T[1] * a0 + T[4] * a1 + T[7] * a2;
            z[3 * i + 2] = T[2] * a0 + T[5] * a1 + T[8] * a2;
        }
    }
}

// u_c = G_c (A_c z) with G_c = s_c (I - qhat qhat^T) (the Delta P blocks)
// dw_mode 1: dL/dw_c += h (A_c z).(p_c - q_c); 2: (A_c z).(p_c - q_c) kept in adj_dwc
template <bool MIXED>
__device__ __forceinline__ void projection_jacobian_apply(const SimDev &S, auto z, auto u, int dw_mode, double h) {
    for (int c = threadIdx.x; c < S.nca; c += (int)blockDim.x) {
        double a0 = 0, a1 = 0, a2 = 0;
        for (int p = G(S.c_ptr)[c]; p < G(S.c_ptr)[c + 1]; ++p) {
            const int j = G(S.c_node)[p];
            const double a = G(S.c_coef)[p];
            a0 += a * z[3 * j];
            a1 += a * z[3 * j + 1];
            a2 += a * z[3 * j + 2];
        }
        const auto qh = G(S.adj_q) + 3 * c;
        if (MIXED) {
            const float sc = (float)G(S.adj_s)[c];
            const float q0 = (float)qh[0], q1 = (float)qh[1], q2 = (float)qh[2];
            const float b0 = (float)a0, b1 = (float)a1, b2 = (float)a2;
            const float qd = q0 * b0 + q1 * b1 + q2 * b2;
            u[3 * c] = (double)(sc * (b0 - qd * q0));
            u[3 * c + 1] = (double)(sc * (b1 - qd * q1));
            u[3 * c + 2] = (double)(sc * (b2 - qd * q2));
        } else {
            const double sc = G(S.adj_s)[c];
            const double qd = qh[0] * a0 + qh[1] * a1 + qh[2] * a2;
            u[3 * c] = sc * (a0 - qd * qh[0]);
            u[3 * c + 1] = sc * (a1 - qd * qh[1]);
            u[3 * c + 2] = sc * (a2 - qd * qh[2]);
        }
        if (dw_mode) {
            const auto pq = G(S.adj_pq) + 3 * c;
            const double dot = a0 * pq[0] + a1 * pq[1] + a2 * pq[2];
            if (dw_mode == 1) G(S.dw)[G(S.c_id)[c]] += h * dot;
            else G(S.adj_dwc)[c] = dot;
        }
    }
}

// dL/dw for constraints without a local projection (flat bending): p = 0.
__device__ __forceinline__ void inactive_dw(const SimDev &S, auto z, auto x1, double h) {
    for (int c = S.nca + threadIdx.x; c < S.nc_total; c += (int)blockDim.x) {
        double a0 = 0, a1 = 0, a2 = 0, q0 = 0, q1 = 0, q2 = 0;
        for (int p = G(S.c_ptr)[c]; p < G(S.c_ptr)[c + 1]; ++p) {
            const int j = G(S.c_node)[p];
            const double a = G(S.c_coef)[p];
            a0 += a * z[3 * j]; a1 += a * z[3 * j + 1]; a2 += a * z[3 * j + 2];
            q0 += a * x1[3 * j]; q1 += a * x1[3 * j + 1]; q2 += a * x1[3 * j + 2];
        }
        G(S.dw)[G(S.c_id)[c]] -= h * (a0 * q0 + a1 * q1 + a2 * q2);
    }
}

// r_i = g_i + sum_c a_ci u_c + h^2 (K_s d)_i, d = zeta - z (FP32 matrix values in mixed mode)
template <bool MIXED>
__device__ __forceinline__ void adjoint_rhs(const SimDev &S, auto gbar, auto u, auto zeta, auto z, auto r) {
    const double hh = S.h * S.h;
    for (int i = threadIdx.x; i < S.m; i += (int)blockDim.x) {
        double r0 = 0, r1 = 0, r2 = 0;
        for (int p = G(S.inc_ptr)[i]; p < G(S.inc_ptr)[i + 1]; ++p) {
            const int c = G(S.inc_con)[p];
            const double a = G(S.inc_coef)[p];
            r0 += a * u[3 * c]; r1 += a * u[3 * c + 1]; r2 += a * u[3 * c + 2];
        }
        double k0 = 0, k1 = 0, k2 = 0;
        for (int p = G(S.ks_ptr)[i]; p < G(S.ks_ptr)[i + 1]; ++p) {
            const int j = G(S.ks_col)[p];
            const double kv = MIXED ? (double)G(S.ks_valf)[p] : G(S.ks_val)[p];
            k0 += kv * (zeta[3 * j] - z[3 * j]);
            k1 += kv * (zeta[3 * j + 1] - z[3 * j + 1]);
            k2 += kv * (zeta[3 * j + 2] - z[3 * j + 2]);
        }
        r[3 * i] = gbar[3 * i] + r0 + hh * k0;
        r[3 * i + 1] = gbar[3 * i + 1] + r1 + hh * k1;
        r[3 * i + 2] = gbar[3 * i + 2] + r2 + hh * k2;
    }
}

// out = A v = M v + H T^T v with H = h^2 K_s - Delta P (the contact adjoint operator).
// KEEP: also keep H z (adj_hz) and the weight-gradient dot products (adj_dwc)
// of z = T^T v, which the step's gradients reuse (z and ΔP z stay in zt, wp).
template <bool MIXED, bool KEEP = false>
__device__ __forceinline__ void apply_adjoint_operator(const SimDev &S, auto mode, auto prt, auto vin, auto out) {
    apply_TT(S, mode, prt, vin, G(S.zt));
    __syncthreads();
    projection_jacobian_apply<MIXED>(S, G(S.zt), G(S.wp), KEEP ? 2 : 0, S.h);
    __syncthreads();
    const double hh = S.h * S.h;
    for (int i = threadIdx.x; i < S.m; i += (int)blockDim.x) {
        double r0 = 0, r1 = 0, r2 = 0;
        for (int p = G(S.inc_ptr)[i]; p < G(S.inc_ptr)[i + 1]; ++p) {
            const int c = G(S.inc_con)[p];
            const double a = G(S.inc_coef)[p];
            r0 += a * G(S.wp)[3 * c]; r1 += a * G(S.wp)[3 * c + 1]; r2 += a * G(S.wp)[3 * c + 2];
        }
        double k0 = 0, k1 = 0, k2 = 0;
        for (int p = G(S.ks_ptr)[i]; p < G(S.ks_ptr)[i + 1]; ++p) {
            const int j = G(S.ks_col)[p];
            const double kv = MIXED ? (double)G(S.ks_valf)[p] : G(S.ks_val)[p];
            k0 += kv * G(S.zt)[3 * j]; k1 += kv * G(S.zt)[3 * j + 1]; k2 += kv * G(S.zt)[3 * j + 2];
        }
        const double mi = G(S.mass)[i];
        out[3 * i] = mi * vin[3 * i] + hh * k0 - r0;
        out[3 * i + 1] = mi * vin[3 * i + 1] + hh * k1 - r1;
        out[3 * i + 2] = mi * vin[3 * i + 2] + hh * k2 - r2;
        if constexpr (KEEP) {
            G(S.adj_hz)[3 * i] = hh * k0 - r0;
            G(S.adj_hz)[3 * i + 1] = hh * k1 - r1;
            G(S.adj_hz)[3 * i + 2] = hh * k2 - r2;
        }
    }
    __syncthreads();
}

// Block-wide dot products <V_k, w> for k = 0..nk-1 (fixed order); results in
// hk[0..nk).  Eight basis vectors per pass over w.
__device__ __forceinline__ void block_dots(auto V, int64_t ld, int nk, auto w, int n3, double *red2, double *hk) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int k0 = 0; k0 < nk; k0 += 8) {
        double p[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        const int kn = min(8, nk - k0);
        for (int i = threadIdx.x; i < n3; i += (int)blockDim.x) {
            const double wi = w[i];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q < kn) p[q] += V[(k0 + q) * ld + i] * wi;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            double v = p[q];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0 && q < kn) red2[wave * (kKryM + 1) + k0 + q] = v;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nk; k += (int)blockDim.x) {
        double s = 0.0;
        for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) s += red2[wv * (kKryM + 1) + k];
        hk[k] = s;
    }
    __syncthreads();
}

// Restarted GMRES(kKryM), left-preconditioned by the prefactored P, for
// (M + H T^T) zeta = gbar; fallback when the paper's fixed point stalls or
// diverges.  Stops when |P^{-1}(gbar - A zeta)| <= tol |P^{-1} gbar|.
// Returns the number of Krylov iterations, negative if the tolerance was missed.
template <bool MIXED>
__device__ __forceinline__ int gmres_solve(const SimDev &S, auto mode, auto prt, auto gbar, auto zeta, double tol, int max_iters,
                           double *red, auto T, auto Y, auto U) {
    __shared__ double Hs[(kKryM + 1) * kKryM];
    __shared__ double cs[kKryM], sn[kKryM], gv[kKryM + 1], yk[kKryM + 1];
    __shared__ double red2[(kBlock / 64) * (kKryM + 1)];
    __shared__ int flag[2];
    const int n3 = 3 * S.m;
    const int64_t ld = n3;
    auto V = G(S.kry);
    double beta0 = -1.0;
    int total = 0;
    for (int i = threadIdx.x; i < n3; i += (int)blockDim.x) zeta[i] = 0.0;
    __syncthreads();
    while (true) {
        // r = P^{-1}(gbar - A zeta)
        apply_adjoint_operator<MIXED>(S, mode, prt, zeta, G(S.rhs));
        for (int i = threadIdx.x; i < n3; i += (int)blockDim.x) G(S.rhs)[i] = gbar[i] - G(S.rhs)[i];
        __syncthreads();
        solve_P(S, G(S.lvl_team_adj), G(S.rhs), T, Y, V, U);
        double ss = 0.0;
        for (int i = threadIdx.x; i < n3; i += (int)blockDim.x) ss += V[i] * V[i];
        const double beta = sqrt(block_sum(ss, red));
        if (beta0 < 0) beta0 = beta;
        if (!(beta > tol * beta0) || !(beta == beta)) return (beta == beta) ? total : -total - 1;
        if (total >= max_iters) return -total - 1;
        for (int i = threadIdx.x; i < n3; i += (int)blockDim.x) V[i] /= beta;
        if (threadIdx.x == 0) {
            gv[0] = beta;
            for (int k = 1; k <= S.kry_m; ++k) gv[k] = 0.0;
        }
        __syncthreads();
        int jdone = 0;
        for (int j = 0; j < S.kry_m; ++j) {
            auto w = V + (j + 1) * ld;
            apply_adjoint_operator<MIXED>(S, mode, prt, V + j * ld, G(S.rhs));
            solve_P(S, G(S.lvl_team_adj), G(S.rhs), T, Y, w, U);
            // classical Gram-Schmidt; a second pass only when the first one
            // cancelled most of w (|w| dropped below 0.7 of its norm)
            double ws = 0.0;
            for (int i = threadIdx.x; i < n3; i += (int)blockDim.x) ws += w[i] * w[i];
            double wn = sqrt(block_sum(ws, red));
            for (int pass = 0; pass < 2; ++pass) {
                block_dots(V, ld, j + 1, w, n3, red2, yk);
                for (int i = threadIdx.x; i < n3; i += (int)blockDim.x) {
                    double acc = w[i];
                    for (int k = 0; k <= j; ++k) acc -= yk[k] * V[k * ld + i];
                    w[i] = acc;
                }
                if (threadIdx.x == 0)
                    for (int k = 0; k <= j; ++k) Hs[k * kKryM + j] = (pass ? Hs[k * kKryM + j] : 0.0) + yk[k];
                __syncthreads();
                ws = 0.0;
                for (int i = threadIdx.x; i < n3; i += (int)blockDim.x) ws += w[i] * w[i];
                const double wa = sqrt(block_sum(ws, red));
                const bool again = wa < 0.7 * wn;
                wn = wa;
                if (!again) break;
            }
            const double hn = wn;
            if (hn > 0)
                for (int i = threadIdx.x; i < n3; i += (int)blockDim.x) w[i] /= hn;
            if (threadIdx.x == 0) {
                // apply previous rotations to column j, then a new one
                for (int k = 0; k < j; ++k) {
                    const double a = Hs[k * kKryM + j], b = Hs[(k + 1) * kKryM + j];
                    Hs[k * kKryM + j] = cs[k] * a + sn[k] * b;
                    Hs[(k + 1) * kKryM + j] = -sn[k] * a + cs[k] * b;
                }
                const double a = Hs[j * kKryM + j], b = hn;
                const double r = sqrt(a * a + b * b);
                cs[j] = r > 0 ? a / r : 1.0;
                sn[j] = r > 0 ? b / r : 0.0;
                Hs[j * kKryM + j] = r;
                Hs[(j + 1) * kKryM + j] = 0.0;
                gv[j + 1] = -sn[j] * gv[j];
                gv[j] = cs[j] * gv[j];
                flag[0] = (fabs(gv[j + 1]) <= tol * beta0 || !(hn > 0)) ? 1 : 0;
            }
            __syncthreads();
            ++total;
            jdone = j + 1;
            if (flag[0] || total >= max_iters) break;
        }
        // y = R^{-1} g, zeta += V y
        if (threadIdx.x == 0) {
            for (int k = jdone - 1; k >= 0; --k) {
                double acc = gv[k];
                for (int l = k + 1; l < jdone; ++l) acc -= Hs[k * kKryM + l] * yk[l];
                yk[k] = acc / Hs[k * kKryM + k];
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n3; i += (int)blockDim.x) {
            double acc = zeta[i];
            for (int k = 0; k < jdone; ++k) acc += yk[k] * V[k * ld + i];
            zeta[i] = acc;
        }
        __syncthreads();
    }
}

// Backward over steps [step_begin, step_end) in reverse, one handle per workgroup.

// ------------------------------------------------------------------ direct adjoint
// Each adjoint step solves A zeta = gbar with A = M + H T^T (H = h^2 K_s (x) I_3
// - Delta P at x_{n+1}, T the contact Jacobian blocks; Sec. 4.2).  The paper
// solves it by a fixed point with the prefactored P and falls back to a direct
// solve; here every step's A is factored up front, all steps at once (one
// workgroup each), on the supernodes of P at the level of degrees of freedom
// (left-looking, children first).  Supernode s keeps D_s^{-1} (its diagonal
// block after the Schur updates, inverted by Gauss-Jordan with row pivoting
// inside the block), B_s = A(R_s, s) and V_s = D_s^{-1} A(s, R_s); the Schur
// update of descendant d onto the blocks it reaches is B_d V_d.

constexpr int kFacBlock = 256;        // threads per factorisation workgroup

__device__ __forceinline__ void contact_T(const SimDev &S, uint8_t md, int o, auto xi, auto ub, double *T) {
    // T = d v / d ubar of the contact update, row-major (identity off contact)
    for (int e = 0; e < 9; ++e) T[e] = (md == STICK) ? 0.0 : ((e % 4 == 0) ? 1.0 : 0.0);
    if (md != SLIP) return;
    double nrm[3], phi;
    contact_frame(S, o, xi, nrm, phi);
    const double mu = S.obst[o].mu, h = S.h;
    const double un = nrm[0] * ub[0] + nrm[1] * ub[1] + nrm[2] * ub[2];
    const double a = un + phi / h;
    double t[3] = {ub[0] - un * nrm[0], ub[1] - un * nrm[1], ub[2] - un * nrm[2]};
    const double tau = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    t[0] /= tau; t[1] /= tau; t[2] /= tau;
    const double sl = mu * (-a) / tau;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            T[3 * r + c] = (1 - sl) * ((r == c ? 1.0 : 0.0) - nrm[r] * nrm[c]) + sl * t[r] * t[c] + mu * t[r] * nrm[c];
}

// Workspace of a factor slot: T blocks (9 m), projection scale + direction
// (4 nca), |A|_inf (1), perturbed pivots per supernode (ns int32).
__device__ __forceinline__ auto slot_ws(const SimDev &S, int slot) {
    return G(S.af_ws) + (int64_t)slot * S.af_ws_size;
}
__device__ __forceinline__ int64_t ws_anorm(const SimDev &S) { return 9 * (int64_t)S.m + 4 * (int64_t)max(S.nca, 1); }

// Assembly of one step's A into its factor slot, one workgroup per (handle,
// slot) pair of work (NULL: handle 0, slot = block index); slot k holds step
// af_step0 + k.  The blocks are stored transposed (see capi: ks_dst).
__global__ __launch_bounds__(kFacBlock) void k_adj_assemble(const SimDev *__restrict__ sims,
                                                            const int32_t *__restrict__ work) {
    const int hidx = work ? work[2 * blockIdx.x] : 0;
    const int slot = work ? work[2 * blockIdx.x + 1] : (int)blockIdx.x;
    const SimDev &S = sims[hidx];
    const int tid = threadIdx.x, bd = blockDim.x;
    const int m = S.m;
    const double hh = S.h * S.h;
    const int rs = S.af_step0 + slot - S.rec_step0;
    const auto x0 = G(S.rec_x) + (int64_t)rs * 3 * m;
    const auto x1 = x0 + 3 * m;
    const auto mode = G(S.rec_mode) + (int64_t)rs * m;
    const auto obst = G(S.rec_obst) + (int64_t)rs * m;
    const auto ubr = G(S.rec_ubar) + (int64_t)rs * 3 * m;
    const auto F = G(S.af) + (int64_t)slot * S.af_size;
    const auto ws = slot_ws(S, slot);
    const auto Tb = ws;
    const auto Gc = ws + 9 * (int64_t)m;
    __shared__ double red[kFacBlock / 64];

    for (int64_t e = tid; e < S.af_size; e += bd) F[e] = 0.0;
    for (int c = tid; c < S.nca; c += bd) {           // projection Jacobians at x_{n+1}
        double q0 = 0, q1 = 0, q2 = 0;
        for (int p = G(S.c_ptr)[c]; p < G(S.c_ptr)[c + 1]; ++p) {
            const int j = G(S.c_node)[p];
            const double a = G(S.c_coef)[p];
            q0 += a * x1[3 * j]; q1 += a * x1[3 * j + 1]; q2 += a * x1[3 * j + 2];
        }
        const double nq = sqrt(q0 * q0 + q1 * q1 + q2 * q2);
        const double rho = G(S.c_rho)[c];
        if (nq < 1e-12 * rho) {
            Gc[4 * c] = 0.0; Gc[4 * c + 1] = 0.0; Gc[4 * c + 2] = 0.0; Gc[4 * c + 3] = 0.0;
        } else {
            Gc[4 * c] = hh * G(S.c_w)[c] * rho / nq;
            Gc[4 * c + 1] = q0 / nq; Gc[4 * c + 2] = q1 / nq; Gc[4 * c + 3] = q2 / nq;
        }
    }
    for (int i = tid; i < m; i += bd) {
        double T[9];
        contact_T(S, mode[i], obst[i], x0 + 3 * i, ubr + 3 * i, T);
        for (int e = 0; e < 9; ++e) Tb[9 * (int64_t)i + e] = T[e];
    }
    __syncthreads();
    // the thread of row i owns every block (i, j)
    double anorm = 0.0;
    for (int i = tid; i < m; i += bd) {
        double rsum[3] = {0.0, 0.0, 0.0};
        for (int e = G(S.ks_ptr)[i]; e < G(S.ks_ptr)[i + 1]; ++e) {
            const auto d = F + G(S.ks_dst)[e];
            const int ld = G(S.ks_ld)[e];
            const double k = hh * G(S.ks_val)[e];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) d[c * ld + r] = r == c ? k : 0.0;
        }
        for (int p = G(S.inc_ptr)[i]; p < G(S.inc_ptr)[i + 1]; ++p) {
            const int c = G(S.inc_con)[p];
            const double sc = Gc[4 * c];
            if (sc == 0.0) continue;
            const double qh[3] = {Gc[4 * c + 1], Gc[4 * c + 2], Gc[4 * c + 3]};
            const double ai = G(S.inc_coef)[p] * sc;
            const int q0 = G(S.c_ptr)[c], q1 = G(S.c_ptr)[c + 1], e0 = G(S.dp_ptr)[p];
            for (int q = q0; q < q1; ++q) {
                const double f = ai * G(S.c_coef)[q];
                const int e = G(S.dp_ks)[e0 + q - q0];
                const auto d = F + G(S.ks_dst)[e];
                const int ld = G(S.ks_ld)[e];
                for (int r = 0; r < 3; ++r)
                    for (int cc = 0; cc < 3; ++cc) d[cc * ld + r] -= f * ((r == cc ? 1.0 : 0.0) - qh[r] * qh[cc]);
            }
        }
        for (int e = G(S.ks_ptr)[i]; e < G(S.ks_ptr)[i + 1]; ++e) {
            const int j = G(S.ks_col)[e];
            const uint8_t md = mode[j];
            const auto d = F + G(S.ks_dst)[e];
            const int ld = G(S.ks_ld)[e];
            double b[9];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) b[3 * r + c] = d[c * ld + r];
            if (md == STICK) {
                for (int q = 0; q < 9; ++q) b[q] = 0.0;
            } else if (md == SLIP) {                      // H_ij T_j^T
                const auto T = Tb + 9 * (int64_t)j;
                double o[9];
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c)
                        o[3 * r + c] = b[3 * r] * T[3 * c] + b[3 * r + 1] * T[3 * c + 1] + b[3 * r + 2] * T[3 * c + 2];
                for (int q = 0; q < 9; ++q) b[q] = o[q];
            }
            if (i == j) {
                const double mi = G(S.mass)[i];
                b[0] += mi; b[4] += mi; b[8] += mi;
            }
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) {
                    d[c * ld + r] = b[3 * r + c];
                    rsum[r] += fabs(b[3 * r + c]);
                }
        }
        anorm = fmax(anorm, fmax(rsum[0], fmax(rsum[1], rsum[2])));
    }
    anorm = block_max(anorm, red);
    if (tid == 0) ws[ws_anorm(S)] = anorm;
}

// Gauss-Jordan inverse in place of the N x N row-major block D (N <= 16 E,
// 256 threads), held in registers: thread (ty, tx) owns entries
// (ty + 16a, tx + 16b).  Pivot rows are chosen by magnitude among the rows not
// used yet, without swapping rows (pivoting inside the block); with p_k the
// pivot row of column k, the array ends as X with inverse[k][p_j] = X[p_k][j],
// which the write-back applies.  Pivots below 1e-13 of the block's largest
// entry are raised to that floor; returns how many.  Two barriers per column.
constexpr int kGjMax = 128;           // largest block (degrees of freedom)
struct GjShared {
    double col[2][kGjMax];
    double row[kGjMax];
    int pk[kGjMax], inv[kGjMax];
};
template <int E>
__device__ __forceinline__ int gj_inverse_regs(GLOBAL double *D, int N, int ld, GjShared *sh, double *red) {
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15, lane = tid & 63;
    double X[E][E];
    double dm = 0.0;
#pragma unroll
    for (int a = 0; a < E; ++a)
#pragma unroll
        for (int b = 0; b < E; ++b) {
            const int i = ty + 16 * a, j = tx + 16 * b;
            X[a][b] = (i < N && j < N) ? D[(int64_t)i * ld + j] : 0.0;
            dm = fmax(dm, fabs(X[a][b]));
        }
    const double floor_ = 1e-13 * block_max(dm, red);
    bool used0 = false, used1 = false;      // rows lane and lane + 64, tracked by every wave alike
    int pert = 0;
    for (int k = 0; k < N; ++k) {
        double *colk = sh->col[k & 1];
        const int bk = k >> 4;
        if (tx == (k & 15)) {
#pragma unroll
            for (int a = 0; a < E; ++a) {
                double v = 0.0;
#pragma unroll
                for (int b = 0; b < E; ++b) v = b == bk ? X[a][b] : v;
                if (ty + 16 * a < N) colk[ty + 16 * a] = v;
            }
        }
        __syncthreads();
        double best = (lane < N && !used0) ? fabs(colk[lane]) : -1.0;
        int bi = lane;
        const double v1 = (lane + 64 < N && !used1) ? fabs(colk[lane + 64]) : -1.0;
        if (v1 > best) { best = v1; bi = lane + 64; }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(best, o, 64);
            const int oi = __shfl_xor(bi, o, 64);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        const int p = bi;
        if (p == lane) used0 = true;
        if (p == lane + 64) used1 = true;
        double piv = colk[p];
        if (!(fabs(piv) >= floor_)) {
            piv = piv < 0.0 ? -floor_ : floor_;
            if (!(piv != 0.0)) piv = 1e-300;
            ++pert;
        }
        if (tid == 0) sh->pk[k] = p;
        const int ap = p >> 4;
        if (ty == (p & 15)) {
#pragma unroll
            for (int b = 0; b < E; ++b) {
                double v = 0.0;
#pragma unroll
                for (int a = 0; a < E; ++a) v = a == ap ? X[a][b] : v;
                if (tx + 16 * b < N) sh->row[tx + 16 * b] = v;
            }
        }
        __syncthreads();
        const double pinv = 1.0 / piv;
#pragma unroll
        for (int a = 0; a < E; ++a) {
            const int i = ty + 16 * a;
            const double f = i < N ? colk[i] : 0.0;
#pragma unroll
            for (int b = 0; b < E; ++b) {
                const int j = tx + 16 * b;
                if (i >= N || j >= N) continue;
                if (i == p) X[a][b] = j == k ? pinv : X[a][b] * pinv;
                else X[a][b] = j == k ? -f * pinv : X[a][b] - f * sh->row[j] * pinv;
            }
        }
    }
    for (int i = tid; i < N; i += (int)blockDim.x) sh->inv[sh->pk[i]] = i;
    __syncthreads();
#pragma unroll
    for (int a = 0; a < E; ++a)
#pragma unroll
        for (int b = 0; b < E; ++b) {
            const int i = ty + 16 * a, j = tx + 16 * b;
            if (i < N && j < N) D[(int64_t)sh->inv[i] * ld + sh->pk[j]] = X[a][b];
        }
    __syncthreads();
    return pert;
}

// Schur update of supernode s by descendant d, as a tiled product: target rows
// a and columns b of R_d (from 3 i0 on) with a or b in s, value -= sum_k
// Bt_d[k][a] Vt_d[b][k].  64 x 64 output tiles, k in chunks of 16 staged in
// LDS (tile: 2 x 16 x 64 doubles), a 4 x 4 block of outputs per thread.
__device__ __forceinline__ void schur_update(const SimDev &S, GLOBAL double *F, const auto &q, const auto &ud,
                                             double *tile) {
    const int tid = threadIdx.x;
    const auto &qd = G(S.lu_sup)[ud.d];
    const int Nd = 3 * qd.n, Rd = 3 * qd.r, N = 3 * q.n, n = q.n;
    const int ldnd = qd.ldn, ldrd = qd.ldr, ldn = q.ldn, ldr = q.ldr;
    const auto Bd = F + qd.off + (int64_t)Nd * ldnd;        // Bt_d: Nd x Rd (row stride ldrd)
    const auto Vd = Bd + (int64_t)Nd * ldrd;                // Vt_d: Rd x Nd (row stride ldnd)
    const auto D = F + q.off;
    const auto Bp = D + (int64_t)N * ldn;
    const auto C = Bp + (int64_t)N * ldr;
    const auto rel = G(S.lu_relmap) + ud.map;
    const int a0 = 3 * ud.i0, a1 = 3 * ud.i1;
    double *ta = tile, *tb = tile + 16 * 64;                // ta[k][a], tb[k][b]
    const int tx = tid & 15, ty = tid >> 4;                  // outputs a = a_t + 4 tx + i, b = b_t + 4 ty + j
    for (int at = a0; at < Rd; at += 64)
        for (int bt = a0; bt < Rd; bt += 64) {
            if (at >= a1 && bt >= a1) continue;             // rows and columns both beyond s
            double acc[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
            for (int k0 = 0; k0 < Nd; k0 += 16) {
                for (int e = tid; e < 16 * 64; e += kFacBlock) {
                    const int kk = e >> 6, c = e & 63, k = k0 + kk;
                    ta[e] = (k < Nd && at + c < Rd) ? Bd[(int64_t)k * ldrd + at + c] : 0.0;
                    const int bb = e >> 4, k2 = k0 + (e & 15);
                    tb[(e & 15) * 64 + bb] = (k2 < Nd && bt + bb < Rd) ? Vd[(int64_t)(bt + bb) * ldnd + k2] : 0.0;
                }
                __syncthreads();
#pragma unroll 4
                for (int kk = 0; kk < 16; ++kk) {
                    double va[4], vb[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) va[i] = ta[kk * 64 + 4 * tx + i];
#pragma unroll
                    for (int j = 0; j < 4; ++j) vb[j] = tb[kk * 64 + 4 * ty + j];
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j) acc[i][j] += va[i] * vb[j];
                }
                __syncthreads();
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int aa = at + 4 * tx + i, bb = bt + 4 * ty + j;
                    if (aa >= Rd || bb >= Rd || (aa >= a1 && bb >= a1)) continue;
                    const int ra = rel[aa / 3 - ud.i0], rb = rel[bb / 3 - ud.i0];
                    const int ca = aa % 3, cb = bb % 3;
                    if (bb < a1) {                          // column in s
                        if (ra < n) D[(int64_t)(3 * rb + cb) * ldn + 3 * ra + ca] -= acc[i][j];
                        else Bp[(int64_t)(3 * rb + cb) * ldr + 3 * (ra - n) + ca] -= acc[i][j];
                    } else {                                // row in s, column in R_s
                        C[(int64_t)(3 * (rb - n) + cb) * ldn + 3 * ra + ca] -= acc[i][j];
                    }
                }
        }
}

// V_t = D_t^{-1} A(t, R_t), transposed: Vt = Ct (D^{-1})^T with Ct (R x N) and
// the stored inverse (D^{-1})^T (N x N), in place over Ct: 64-row bands of Ct,
// k in chunks of 16 staged in LDS (tile: 64 x 16 + 16 x 128 doubles), a 4 x 4
// block of outputs per thread and column tile (N <= 128: two column tiles).
__device__ __forceinline__ void v_product(GLOBAL double *C, GLOBAL const double *Dinv, int R, int N, int ld,
                                          double *tile) {
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    double *ta = tile, *tb = tile + 64 * 16;                // ta[k][j], tb[k][i]
    for (int jb = 0; jb < R; jb += 64) {
        double acc[2][4][4];
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[c][i][j] = 0.0;
        for (int k0 = 0; k0 < N; k0 += 16) {
            for (int e = tid; e < 64 * 16; e += kFacBlock) {
                const int jj = e >> 4, kk = e & 15;
                ta[kk * 64 + jj] = (jb + jj < R && k0 + kk < N) ? C[(int64_t)(jb + jj) * ld + k0 + kk] : 0.0;
            }
            for (int e = tid; e < 16 * 128; e += kFacBlock) {
                const int kk = e >> 7, ii = e & 127;
                tb[e] = (k0 + kk < N && ii < N) ? Dinv[(int64_t)(k0 + kk) * ld + ii] : 0.0;
            }
            __syncthreads();
#pragma unroll 4
            for (int kk = 0; kk < 16; ++kk) {
                double va[4], vb[2][4];
#pragma unroll
                for (int j = 0; j < 4; ++j) va[j] = ta[kk * 64 + 4 * ty + j];
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int i = 0; i < 4; ++i) vb[c][i] = tb[kk * 128 + 64 * c + 4 * tx + i];
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int i = 0; i < 4; ++i) acc[c][j][i] += va[j] * vb[c][i];
            }
            __syncthreads();
        }
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = jb + 4 * ty + j, col = 64 * c + 4 * tx + i;
                    if (row < R && col < N) C[(int64_t)row * ld + col] = acc[c][j][i];
                }
        __syncthreads();
    }
}

// One workgroup per (handle, slot, chunk) of one level of the factor's tree:
// the Schur updates of the descendants reaching the chunk (finished by earlier
// launches), the Gauss-Jordan inverse of its diagonal block (E x E register
// tile per thread, N <= 16 E), then V.  Blocks are stored transposed: Dt = D^T,
// Bt = B^T (N x R), Ct = A(t, R_t)^T (R x N), row-major.
constexpr int kFacTile = 64 * 16 + 16 * 128;                 // doubles of LDS for the product tiles
template <int E>
__global__ __launch_bounds__(kFacBlock) void k_adj_factor_level(const SimDev *__restrict__ sims,
                                                                const int32_t *__restrict__ work) {
    const int hidx = work[3 * blockIdx.x], slot = work[3 * blockIdx.x + 1], sn = work[3 * blockIdx.x + 2];
    const SimDev &S = sims[hidx];
    const auto F = G(S.af) + (int64_t)slot * S.af_size;
    const auto ws = slot_ws(S, slot);
    __shared__ double tile[kFacTile];
    __shared__ GjShared small;
    __shared__ double red[kFacBlock / 64];
    const auto &q = G(S.lu_sup)[sn];
    const int N = 3 * q.n, R = 3 * q.r;
    const auto D = F + q.off;
    const auto C = D + (int64_t)N * q.ldn + (int64_t)N * q.ldr;
    for (int u = G(S.lu_upd_ptr)[sn]; u < G(S.lu_upd_ptr)[sn + 1]; ++u) {
        schur_update(S, F, q, G(S.lu_upd)[u], tile);
        __syncthreads();
    }
    const int pert = gj_inverse_regs<E>(D, N, q.ldn, &small, red);
    if (R > 0) v_product(C, D, R, N, q.ldn, tile);
    if (threadIdx.x == 0) ((GLOBAL int32_t *)(ws + ws_anorm(S) + 1))[sn] = pert;
}

// lane j's value of x, for every lane (j wave-uniform)
__device__ __forceinline__ double lane_value(double x, int j) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), j);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// the solving workgroup announces the phase it starts (pos: step * phases + phase)
__device__ __forceinline__ void publish_pos(const SimDev &S, int64_t pos) { announce(S.adj_pos, S.adj_epoch, pos); }

// One phase of the direct adjoint solve (see AdjItem): every wavefront runs
// its share of the column batches, two rows per lane (one 16-byte load per
// column), the columns of a short item split over groups of lanes and summed
// in a fixed tree; an item finished inside the share is written at once, a
// part of an item that spans several wavefronts goes to part[] and is
// summed, in wavefront order, after the barrier.
// OP 0: out = M v; OP 1: out = z - M v.
template <int OP>
__device__ __forceinline__ void adj_phase(const SimDev &S, int ph, auto F, auto v, auto z, auto out, double *part) {
    constexpr bool kGlobalV = !std::is_same_v<decltype(v), double *>;   // v not in LDS
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const auto items = (GLOBAL const v4i *)S.adj_items;                 // AdjItem as 2 x 16 bytes
    const auto F2 = (GLOBAL const v2d *)F;                               // step factors: even offsets
    const v4i pr = ((GLOBAL const v4i *)S.adj_prog)[ph * kAdjWaves + wave];
    int i = pr.x, kb = pr.y;
    while (i < pr.z || (i == pr.z && kb < pr.w)) {
        const v4i d0 = items[2 * i], d1 = items[2 * i + 1];
        const int64_t moff = (int64_t)(uint32_t)d0.x | ((int64_t)d0.y << 32);
        const int ld2 = d0.z >> 1, K = d0.w, vb = d1.x, ob = d1.y, nrow = d1.z, ng = d1.w;
        // lane = g rp + rr: rows 2 rr, 2 rr + 1; column group g of ng
        const int rp = (nrow + 1) >> 1, g = lane / rp, rr = lane - g * rp, r0 = 2 * rr;
        const bool grp_ok = g < ng, live = grp_ok && r0 < nrow;
        const int span = kAdjBatch * ng;
        const int nkb = K > 0 ? (K + span - 1) / span : 1;
        const int kend = i == pr.z ? pr.w : nkb;
        const bool whole = kb == 0 && kend == nkb;
        const auto col = F2 + ((moff >> 1) + rr);
        double acc0 = 0.0, acc1 = 0.0;
        for (; kb < kend; ++kb) {
            const int k0 = kb * span, kg = k0 + g * kAdjBatch;
            v2d c[kAdjBatch];
            if (k0 + span <= K) {                       // full batch: one predicate for all loads
                // v in global memory: one load by lanes 0..span-1, read back from registers
                double vl = 0.0;
                if constexpr (kGlobalV)
                    if (lane < span) vl = v[vb + k0 + lane];
                if (live) {
#pragma unroll
                    for (int j = 0; j < kAdjBatch; ++j) c[j] = col[(kg + j) * ld2];
                } else {
#pragma unroll
                    for (int j = 0; j < kAdjBatch; ++j) c[j] = v2d{0.0, 0.0};
                }
#pragma unroll
                for (int j = 0; j < kAdjBatch; ++j) {
                    double vj;
                    if constexpr (kGlobalV) vj = ng == 1 ? lane_value(vl, j) : __shfl(vl, g * kAdjBatch + j, 64);
                    else vj = grp_ok ? v[vb + kg + j] : 0.0;
                    acc0 += c[j].x * vj;
                    acc1 += c[j].y * vj;
                }
            } else {
#pragma unroll
                for (int j = 0; j < kAdjBatch; ++j)
                    c[j] = live && kg + j < K ? col[(kg + j) * ld2] : v2d{0.0, 0.0};
#pragma unroll
                for (int j = 0; j < kAdjBatch; ++j)
                    if (grp_ok && kg + j < K) {
                        const double vj = v[vb + kg + j];
                        acc0 += c[j].x * vj;
                        acc1 += c[j].y * vj;
                    }
            }
        }
        for (int sft = ng >> 1; sft > 0; sft >>= 1) {   // groups summed in a fixed tree; group 0 holds the row sums
            acc0 += __shfl_down(acc0, sft * rp, 64);
            acc1 += __shfl_down(acc1, sft * rp, 64);
        }
        if (g == 0) {
            if (whole) {
                if (r0 < nrow) out[ob + r0] = OP == 0 ? acc0 : z[ob + r0] - acc0;
                if (r0 + 1 < nrow) out[ob + r0 + 1] = OP == 0 ? acc1 : z[ob + r0 + 1] - acc1;
            } else {
                const int o = (2 * wave + (i == pr.x ? 0 : 1)) * kAdjRows + r0;
                part[o] = acc0;
                part[o + 1] = acc1;
            }
        }
        ++i;
        kb = 0;
    }
    __syncthreads();
    const int s0 = G(S.adj_sptr)[ph], s1 = G(S.adj_sptr)[ph + 1];
    if (s1 > s0) {
        const int r0 = 2 * lane;                         // parts are stored by row
        for (int e = s0 + wave; e < s1; e += kAdjWaves) {
            const v4i sp = ((GLOBAL const v4i *)S.adj_split)[e];
            const v4i d1 = items[2 * sp.x + 1];
            double acc0 = 0.0, acc1 = 0.0;
            for (int w = sp.y; w <= sp.z; ++w) {
                const v4i pw = ((GLOBAL const v4i *)S.adj_prog)[ph * kAdjWaves + w];
                if (pw.x == pw.z && pw.y == pw.w) continue;          // empty run: no part
                const int o = (2 * w + (sp.x == pw.x ? 0 : 1)) * kAdjRows + r0;
                acc0 += part[o];
                acc1 += part[o + 1];
            }
            const int ob = d1.y, nrow = d1.z;
            if (r0 < nrow) out[ob + r0] = OP == 0 ? acc0 : z[ob + r0] - acc0;
            if (r0 + 1 < nrow) out[ob + r0 + 1] = OP == 0 ? acc1 : z[ob + r0 + 1] - acc1;
        }
        __syncthreads();
    }
}

// x = A^{-1} b with a step factor F: forward sweep by level (gather t_t,
// z_t = D_t^{-1} t_t, u_t = B_t z_t), backward sweep (gather x_{R_t},
// x_t = z_t - V_t x_{R_t}).  T, Z, U: work vectors; part: 2 x kAdjRows doubles per wavefront.
__device__ __forceinline__ void solve_A(const SimDev &S, auto F, auto b, auto T, auto Z, auto x, auto U,
                                        double *part, int64_t pos0) {
    const int tid = threadIdx.x, bd = blockDim.x;
    const auto lvl = G(S.lu_lvl);
    const int L = S.lu_nlevels;
    for (int l = 0; l < L; ++l) {
        publish_pos(S, pos0 + 2 * l);
        gather_rows(G(S.lu_rows), G(S.lu_upd_off), lvl[2 * l], lvl[2 * (l + 1)], b, T, U);
        __syncthreads();
        adj_phase<0>(S, 3 * l, F, T, Z, Z, part);
        publish_pos(S, pos0 + 2 * l + 1);
        adj_phase<0>(S, 3 * l + 1, F, Z, Z, U, part);
    }
    for (int l = L - 1; l >= 0; --l) {
        publish_pos(S, pos0 + 2 * L + (L - 1 - l));
        const int q0 = lvl[2 * l + 1], q1 = lvl[2 * (l + 1) + 1];
        if (q1 > q0) {
            for (int q = q0 + tid; q < q1; q += bd) {
                const v2i e = ((GLOBAL const v2i *)S.lu_gat)[q];   // GatherItem {u, x3}
                U[e.x] = x[e.y]; U[e.x + 1] = x[e.y + 1]; U[e.x + 2] = x[e.y + 2];
            }
            __syncthreads();
        }
        adj_phase<1>(S, 3 * l + 2, F, U, Z, x, part);
    }
}

// Helper workgroup j of H (same XCD as the solving workgroup): walks the
// phases of the launch's steps in the solver's order and touches every
// 128-byte line of the blocks a phase reads (one load per line, results
// discarded), at most one phase ahead of the solver's published position.  It
// only reads; it stops when the solver is done, or when no new position has
// arrived for 100 ms.
__device__ void adj_prefetch(const SimDev &S, int j, int H) {
    __shared__ int go;
    const int L = S.lu_nlevels, PH = 3 * L;
    const int64_t stride = (int64_t)H * blockDim.x;
    const int64_t me = (int64_t)j * blockDim.x + threadIdx.x;
    uint64_t sink = 0;
    for (int k = 0; k < S.step_end - S.step_begin; ++k) {
        const int n = S.step_end - 1 - k;
        const auto F = G(S.af) + (int64_t)(n - S.af_step0) * S.af_size;
        for (int q = 0; q < PH; ++q) {
            const int64_t target = (int64_t)k * PH + q;
            if (threadIdx.x == 0) {
                int state = 0;                                   // 0: give up, 1: go, 2: solver done
                const uint64_t t0 = wall_clock64();
                while (wall_clock64() - t0 < 10000000ull) {      // 100 ms at the 100 MHz wall clock
                    const int64_t p = __hip_atomic_load(S.adj_pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if ((p >> 40) == S.adj_epoch) {
                        if ((p & kPosMask) == kPosMask) { state = 2; break; }
                        if ((p & kPosMask) + 1 >= target) { state = 1; break; }
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                go = state;
            }
            __syncthreads();
            const int st = go;
            __syncthreads();
            if (st != 1) {
                if (sink == 0x9e3779b97f4a7c15ull) G(S.red)[63] = 1.0;   // keeps the loads
                return;
            }
            const int ph = q < 2 * L ? 3 * (q >> 1) + (q & 1) : 3 * (L - 1 - (q - 2 * L)) + 2;
            int64_t line0 = 0;                                   // first line of the range in the phase
            for (int r = G(S.adj_pfptr)[ph]; r < G(S.adj_pfptr)[ph + 1]; ++r) {
                const int64_t o = G(S.adj_pf)[2 * r], len = G(S.adj_pf)[2 * r + 1];
                const int64_t nl = (len + 15) / 16;
                int64_t i = (me - line0) % stride;               // lines i of the range with line0 + i = me mod stride
                if (i < 0) i += stride;
                for (; i < nl; i += stride) {
                    sink ^= (uint64_t)__double_as_longlong(F[o + 16 * i]);
                    if (i == nl - 1) sink ^= (uint64_t)__double_as_longlong(F[o + len - 1]);
                }
                line0 += nl;
            }
        }
    }
    if (sink == 0x9e3779b97f4a7c15ull) G(S.red)[63] = 1.0;
}

// Slip block T = dv/dubar = (1 - s)(I - n n^T) + s t t^T + mu t n^T of the
// closed-form law (t the unit free tangential velocity, s = mu(-a)/|u_T|),
// written row-major to T.
__device__ __forceinline__ void slip_block(const double *ub, const double *nrm, double phi, double mu, double h,
                                           GLOBAL double *T) {
    const double un = nrm[0] * ub[0] + nrm[1] * ub[1] + nrm[2] * ub[2];
    const double a = un + phi / h;
    double t[3] = {ub[0] - un * nrm[0], ub[1] - un * nrm[1], ub[2] - un * nrm[2]};
    const double tau = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    t[0] /= tau; t[1] /= tau; t[2] /= tau;
    const double s = mu * (-a) / tau;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            T[3 * r + c] = (1 - s) * ((r == c ? 1.0 : 0.0) - nrm[r] * nrm[c]) + s * t[r] * t[c] + mu * t[r] * nrm[c];
}

// Gradients through the contact frame of an active contact (stick / slip)
// with multiplier lam (M zeta; a pair: its reduced mass times zeta_L - zeta_F):
// dphi = lam^T dv/dphi, dn = (dv/dn)^T lam (ubar and the gap held fixed) and
// lam^T dv/dmu, for v = -(phi/h) n (stick), -(phi/h) n + u_T + mu a t (slip).
__device__ __forceinline__ void frame_grad(const double *lam, const double *nrm, double phi, const double *ub,
                                           double mu, bool slip, double h, double &dphi, double *dn,
                                           double &dmu) {
    const double nl = nrm[0] * lam[0] + nrm[1] * lam[1] + nrm[2] * lam[2];
    dmu = 0.0;
    if (!slip) {
        dphi = -nl / h;
        for (int d = 0; d < 3; ++d) dn[d] = -(phi / h) * lam[d];
        return;
    }
    const double un = nrm[0] * ub[0] + nrm[1] * ub[1] + nrm[2] * ub[2];
    const double a = un + phi / h;
    double t[3] = {ub[0] - un * nrm[0], ub[1] - un * nrm[1], ub[2] - un * nrm[2]};
    const double tau = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    t[0] /= tau; t[1] /= tau; t[2] /= tau;
    const double tl = t[0] * lam[0] + t[1] * lam[1] + t[2] * lam[2];
    dphi = (-nl + mu * tl) / h;
    dmu = a * tl;
    double El[3];
    for (int d = 0; d < 3; ++d) El[d] = (lam[d] - t[d] * tl) / tau;
    const double nE = nrm[0] * El[0] + nrm[1] * El[1] + nrm[2] * El[2];
    for (int d = 0; d < 3; ++d)
        dn[d] = -(phi / h) * lam[d] + (-un * lam[d] - ub[d] * nl) + mu * tl * ub[d] + mu * a * (-un * El[d] - ub[d] * nE);
}

template <bool MIXED, int FL>
__global__ __launch_bounds__(kBlockAdj) void k_backward(const SimDev *__restrict__ sims, int helpers) {
    if (helpers > 0 && blockIdx.x > 0) {                 // single-handle launch: prefetch helpers
        if constexpr ((FL & kAdjDirect) != 0)
            if (blockIdx.x % kXcds == 0 && blockIdx.x / kXcds <= helpers)
                adj_prefetch(sims[0], blockIdx.x / kXcds - 1, helpers);
        return;
    }
    const SimDev &S = sims[blockIdx.x];
    extern __shared__ double dyn[];
    __shared__ double red[kBlock / 64];
    constexpr bool kv = (FL & kLdsVectors) != 0, ku = (FL & kLdsUpdates) != 0;
    constexpr bool direct = (FL & kAdjDirect) != 0;      // per-step factors (else fixed point + GMRES)
    constexpr bool km = (FL & kMeshObst) != 0;
    auto T = pick<kv>(dyn, G(S.rhs));
    auto Y = pick<kv>(dyn + 3 * S.m, G(S.ysol));
    auto U = pick<ku>(dyn + (kv ? 6 * S.m : 0), G(S.ubuf));
    const int m = S.m;
    const double h = S.h, hh = h * h;
    int64_t iters_total = 0, gm_total = 0, pert_total = 0;
    int noconv = 0;
    for (int n = S.step_end - 1; n >= S.step_begin; --n) {
        const int slot = n - S.rec_step0;
        const auto x0 = G(S.rec_x) + (int64_t)slot * 3 * m;
        const auto x1 = x0 + 3 * m;
        const auto mode = G(S.rec_mode) + (int64_t)slot * m;
        const auto obst = G(S.rec_obst) + (int64_t)slot * m;
        const auto prt = G(S.rec_partner) + (S.self_on ? (int64_t)slot * m : 0);
        const auto ubr = G(S.rec_ubar) + (int64_t)slot * 3 * m;
        auto gbar = G(S.b0);
        // projections and their Jacobians at x_{n+1}
        for (int c = threadIdx.x; c < S.nca; c += (int)blockDim.x) {
            double q0 = 0, q1 = 0, q2 = 0;
            for (int p = G(S.c_ptr)[c]; p < G(S.c_ptr)[c + 1]; ++p) {
                const int j = G(S.c_node)[p];
                const double a = G(S.c_coef)[p];
                q0 += a * x1[3 * j]; q1 += a * x1[3 * j + 1]; q2 += a * x1[3 * j + 2];
            }
            const double nq = sqrt(q0 * q0 + q1 * q1 + q2 * q2);
            const double rho = G(S.c_rho)[c];
            double p0, p1, p2, sc, qh0, qh1, qh2;
            if (nq < 1e-12 * rho) {
                p0 = rho * G(S.c_restdir)[3 * c]; p1 = rho * G(S.c_restdir)[3 * c + 1]; p2 = rho * G(S.c_restdir)[3 * c + 2];
                sc = 0.0; qh0 = qh1 = qh2 = 0.0;
            } else {
                qh0 = q0 / nq; qh1 = q1 / nq; qh2 = q2 / nq;
                p0 = rho * qh0; p1 = rho * qh1; p2 = rho * qh2;
                sc = hh * G(S.c_w)[c] * rho / nq;
            }
            G(S.adj_s)[c] = sc;
            G(S.adj_q)[3 * c] = qh0; G(S.adj_q)[3 * c + 1] = qh1; G(S.adj_q)[3 * c + 2] = qh2;
            G(S.adj_pq)[3 * c] = p0 - q0; G(S.adj_pq)[3 * c + 1] = p1 - q1; G(S.adj_pq)[3 * c + 2] = p2 - q2;
        }
        // gbar and the contact blocks T_j (slip)
        for (int i = threadIdx.x; i < m; i += (int)blockDim.x) {
            for (int d = 0; d < 3; ++d) {
                gbar[3 * i + d] = G(S.gv)[3 * i + d] + h * G(S.gx)[3 * i + d];
                G(S.zeta)[3 * i + d] = 0.0;
            }
            if (S.self_on && prt[i] >= 0) {
                // a pair in slip: its relative block T_r, the same in both nodes
                if (mode[i] == SLIP) {
                    const int p = prt[i];
                    const bool lead = G(S.caller_id)[i] < G(S.caller_id)[p];
                    const int L = lead ? i : p, F = lead ? p : i;
                    double nrm[3], phi, r;
                    self_frame(S, L, F, x0, nrm, phi, r);
                    const double ub[3] = {ubr[3 * L] - ubr[3 * F], ubr[3 * L + 1] - ubr[3 * F + 1],
                                          ubr[3 * L + 2] - ubr[3 * F + 2]};
                    slip_block(ub, nrm, phi, S.self_mu, h, G(S.tblk) + 9 * (int64_t)i);
                }
                continue;
            }
            bool cached = false;
            if constexpr (km) {
                // mesh: the frame at x_n (normal, gap, edge direction, region) scanned
                // once per step and node, for the blocks T_j and the gradients
                if ((mode[i] == STICK || mode[i] == SLIP) && S.obst[obst[i]].type == 2) {
                    const double xv[3] = {x0[3 * i], x0[3 * i + 1], x0[3 * i + 2]};
                    double nm[3], pm, em[3];
                    int reg;
                    mesh_frame(S.obst[obst[i]], xv, nm, pm, reg, em);
                    auto cf = G(S.cfr) + 8 * (int64_t)i;
                    for (int d = 0; d < 3; ++d) { cf[d] = nm[d]; cf[4 + d] = em[d]; }
                    cf[3] = pm;
                    cf[7] = (double)reg;
                    cached = true;
                }
            }
            if (mode[i] == SLIP) {
                double nrm[3], phi;
                if (cached) {
                    for (int d = 0; d < 3; ++d) nrm[d] = G(S.cfr)[8 * i + d];
                    phi = G(S.cfr)[8 * i + 3];
                } else {
                    contact_frame<false>(S, obst[i], x0 + 3 * i, nrm, phi);
                }
                const auto ub = ubr + 3 * i;
                const double ubv[3] = {ub[0], ub[1], ub[2]};
                slip_block(ubv, nrm, phi, S.obst[obst[i]].mu, h, G(S.tblk) + 9 * (int64_t)i);
            }
        }
        __syncthreads();
        auto zeta = G(S.zeta);
        auto zeta1 = G(S.zeta1);
        if constexpr (direct) {
            // zeta = A^{-1} gbar with the step's factor, refined against A until the
            // normwise backward error |gbar - A zeta| / (|A| |zeta| + |gbar|) (max
            // norms) is at most adj_tol
            const auto F = G(S.af) + (int64_t)(n - S.af_step0) * S.af_size;
            const auto wsn = slot_ws(S, n - S.af_step0) + ws_anorm(S);
            const double anorm = wsn[0];
            __shared__ double part[kAdjWaves * 2 * kAdjRows];  // parts of split items
            const int64_t pos0 = (int64_t)(S.step_end - 1 - n) * 3 * S.lu_nlevels;
            solve_A(S, F, gbar, T, Y, zeta, U, part, pos0);
            double gmax = 0.0;
            for (int i = threadIdx.x; i < 3 * m; i += (int)blockDim.x) gmax = fmax(gmax, fabs(gbar[i]));
            gmax = block_max(gmax, red);
            int k = 1;
            bool ok = false;
            while (true) {
                apply_adjoint_operator<MIXED, true>(S, mode, prt, zeta, zeta1);
                double rmax = 0.0, zmax = 0.0;
                for (int i = threadIdx.x; i < 3 * m; i += (int)blockDim.x) {
                    zeta1[i] = gbar[i] - zeta1[i];
                    rmax = fmax(rmax, fabs(zeta1[i]));
                    zmax = fmax(zmax, fabs(zeta[i]));
                }
                rmax = block_max(rmax, red);
                zmax = block_max(zmax, red);
                const bool finite = rmax == rmax && zmax == zmax && zmax < 1e300;
                if (finite && !(rmax > S.adj_tol * (anorm * zmax + gmax))) { ok = true; break; }
                if (k >= S.adj_max_iters || !finite) break;
                solve_A(S, F, zeta1, T, Y, G(S.zt), U, part, pos0);
                for (int i = threadIdx.x; i < 3 * m; i += (int)blockDim.x) zeta[i] += G(S.zt)[i];
                __syncthreads();
                ++k;
            }
            iters_total += k;
            if (!ok) ++noconv;
            if (threadIdx.x == 0) {
                const auto pc = (GLOBAL const int32_t *)(wsn + 1);
                for (int q = 0; q < S.ns; ++q) pert_total += pc[q];
            }
        } else {
        // fixed point zeta <- P^{-1}[gbar + dP z + (P - M)(zeta - z)], z = T^T zeta
        int k = 0;
        bool ok = false, stalled = false;
        double dprev = 0.0, d5 = 0.0;
        int rising = 0;
        while (k < S.adj_max_iters) {
            apply_TT(S, mode, prt, zeta, G(S.zt));
            __syncthreads();
            projection_jacobian_apply<MIXED>(S, G(S.zt), G(S.wp), 0, h);
            __syncthreads();
            adjoint_rhs<MIXED>(S, gbar, G(S.wp), zeta, G(S.zt), T);
            __syncthreads();
            solve_P(S, G(S.lvl_team_adj), T, T, Y, zeta1, U);
            double dmax = 0.0, zmax = 0.0;
            for (int i = threadIdx.x; i < 3 * m; i += (int)blockDim.x) {
                dmax = fmax(dmax, fabs(zeta1[i] - zeta[i]));
                zmax = fmax(zmax, fabs(zeta1[i]));
            }
            dmax = block_max(dmax, red);
            zmax = block_max(zmax, red);
            ++k;
            auto tmp = zeta; zeta = zeta1; zeta1 = tmp;
            if (dmax == dmax && zmax == zmax && !(dmax > S.adj_tol * zmax)) { ok = true; break; }
            // divergence (3 rises in a row / non-finite) or a contraction too slow
            // to reach the tolerance within the remaining budget -> fallback
            rising = (dmax > dprev && k > 1) ? rising + 1 : 0;
            dprev = dmax;
            if (!(dmax == dmax) || dmax > 1e300 || rising >= 3) { stalled = true; break; }
            if (k % 10 == 5) d5 = dmax;
            if (k % 10 == 0 && k >= 20) {
                const double rate = pow(dmax / d5, 0.2);
                const double need = log(S.adj_tol * zmax / dmax) / log(rate);
                if (!(rate < 1.0) || need > (double)(S.adj_max_iters - k)) { stalled = true; break; }
            }
        }
        iters_total += k;
        if (!ok) {
            if (threadIdx.x == 0) G(S.counters)[2] += 1;
            const int it = gmres_solve<MIXED>(S, mode, prt, gbar, G(S.zeta), S.adj_tol, S.adj_max_iters, red, T, Y, U);
            zeta = G(S.zeta);
            if (it < 0) ++noconv;
            gm_total += it < 0 ? -it - 1 : it;
            (void)stalled;
        }
        }
        // gradients of this step; the direct solve's last backward-error check
        // (always of the final zeta) left z = T^T zeta in zt, H z in adj_hz and
        // the weight-gradient dot products in adj_dwc
        if constexpr (direct) {
            for (int c = threadIdx.x; c < S.nca; c += (int)blockDim.x) G(S.dw)[G(S.c_id)[c]] += h * G(S.adj_dwc)[c];
            inactive_dw(S, G(S.zt), x1, h);
        } else {
            apply_TT(S, mode, prt, zeta, G(S.zt));
            __syncthreads();
            projection_jacobian_apply<MIXED>(S, G(S.zt), G(S.wp), 1, h);
            inactive_dw(S, G(S.zt), x1, h);
            __syncthreads();
        }
        double dmu_local[kMaxObstacles];
        for (int o = 0; o < kMaxObstacles; ++o) dmu_local[o] = 0.0;
        double dmu_self = 0.0;
        // external force: dL/df_ext,n = h z_n, so dL/dF += h s_n z_n and dL/ds_n = h F . z_n
        const bool has_force = S.fext != nullptr;
        const double fs = has_force && S.fscale != nullptr ? G(S.fscale)[n] : 1.0;
        double fz = 0.0;
        const bool has_gstep = S.gx_steps != nullptr;
        const auto gstep = G(S.gx_steps) + (has_gstep ? (int64_t)n * 3 * m : 0);
        for (int i = threadIdx.x; i < m; i += (int)blockDim.x) {
            const auto z = G(S.zt) + 3 * i;
            double Hz[3];
            if constexpr (direct) {
                Hz[0] = G(S.adj_hz)[3 * i]; Hz[1] = G(S.adj_hz)[3 * i + 1]; Hz[2] = G(S.adj_hz)[3 * i + 2];
            } else {
                double r0 = 0, r1 = 0, r2 = 0;      // Delta P z
                for (int p = G(S.inc_ptr)[i]; p < G(S.inc_ptr)[i + 1]; ++p) {
                    const int c = G(S.inc_con)[p];
                    const double a = G(S.inc_coef)[p];
                    r0 += a * G(S.wp)[3 * c]; r1 += a * G(S.wp)[3 * c + 1]; r2 += a * G(S.wp)[3 * c + 2];
                }
                double k0 = 0, k1 = 0, k2 = 0;      // K_s z
                for (int p = G(S.ks_ptr)[i]; p < G(S.ks_ptr)[i + 1]; ++p) {
                    const int j = G(S.ks_col)[p];
                    const double kv = MIXED ? (double)G(S.ks_valf)[p] : G(S.ks_val)[p];
                    k0 += kv * G(S.zt)[3 * j]; k1 += kv * G(S.zt)[3 * j + 1]; k2 += kv * G(S.zt)[3 * j + 2];
                }
                Hz[0] = hh * k0 - r0; Hz[1] = hh * k1 - r1; Hz[2] = hh * k2 - r2;
            }
            const double mi = G(S.mass)[i];
            double dx[3];
            for (int d = 0; d < 3; ++d) dx[d] = G(S.gx)[3 * i + d] - Hz[d] / h;
            const uint8_t md = mode[i];
            const int pi_ = S.self_on ? prt[i] : -1;
            if (pi_ >= 0 && (md == STICK || md == SLIP)) {
                // pair: multiplier m_LF (zeta_L - zeta_F); phi = |x_L - x_F| - d and
                // n = (x_L - x_F)/r give dphi/dx_L = n, dn/dx_L = (I - n n^T)/r,
                // the negatives for x_F
                const bool lead = G(S.caller_id)[i] < G(S.caller_id)[pi_];
                const int L = lead ? i : pi_, F = lead ? pi_ : i;
                const double mL = G(S.mass)[L], mF = G(S.mass)[F], mred = mL * mF / (mL + mF);
                double nrm[3], phi, r;
                self_frame(S, L, F, x0, nrm, phi, r);
                const double lam[3] = {mred * (zeta[3 * L] - zeta[3 * F]), mred * (zeta[3 * L + 1] - zeta[3 * F + 1]),
                                       mred * (zeta[3 * L + 2] - zeta[3 * F + 2])};
                const double ub[3] = {ubr[3 * L] - ubr[3 * F], ubr[3 * L + 1] - ubr[3 * F + 1],
                                      ubr[3 * L + 2] - ubr[3 * F + 2]};
                double dphi, dn[3], dmt;
                frame_grad(lam, nrm, phi, ub, S.self_mu, md == SLIP, h, dphi, dn, dmt);
                if (lead) dmu_self += dmt;
                const double ndn = nrm[0] * dn[0] + nrm[1] * dn[1] + nrm[2] * dn[2];
                const double sg = lead ? 1.0 : -1.0;
                for (int d = 0; d < 3; ++d) dx[d] += sg * (dphi * nrm[d] + (dn[d] - ndn * nrm[d]) / r);
            } else if (md == STICK || md == SLIP) {
                const int o = obst[i];
                double nrm[3], phi;
                bool cached = false;                         // mesh: the frame scanned for T_j above
                if constexpr (km) cached = S.obst[o].type == 2;
                if (cached) {
                    for (int d = 0; d < 3; ++d) nrm[d] = G(S.cfr)[8 * i + d];
                    phi = G(S.cfr)[8 * i + 3];
                } else {
                    contact_frame<false>(S, o, x0 + 3 * i, nrm, phi);
                }
                const double lam[3] = {mi * zeta[3 * i], mi * zeta[3 * i + 1], mi * zeta[3 * i + 2]};
                const auto ub = ubr + 3 * i;
                const double ubv[3] = {ub[0], ub[1], ub[2]};
                double dphi, dn[3], dmt;
                frame_grad(lam, nrm, phi, ubv, S.obst[o].mu, md == SLIP, h, dphi, dn, dmt);
                dmu_local[o] += dmt;
                for (int d = 0; d < 3; ++d) dx[d] += dphi * nrm[d];
                if (S.obst[o].type == 1) {
                    const double e0 = x0[3 * i] - S.obst[o].p[0], e1 = x0[3 * i + 1] - S.obst[o].p[1],
                                 e2 = x0[3 * i + 2] - S.obst[o].p[2];
                    const double r = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
                    const double ndn = nrm[0] * dn[0] + nrm[1] * dn[1] + nrm[2] * dn[2];
                    for (int d = 0; d < 3; ++d) dx[d] += (dn[d] - ndn * nrm[d]) / r;
                } else if constexpr (km) {
                    if (S.obst[o].type == 2) {
                        // dn/dx of the mesh frame at x_n: 0 on a face, (I - n n^T)/phi at
                        // a vertex, (I - n n^T - e e^T)/phi on an edge; phi = 0: as a face
                        const auto cf = G(S.cfr) + 8 * (int64_t)i;
                        const double nm[3] = {cf[0], cf[1], cf[2]}, pm = cf[3], em[3] = {cf[4], cf[5], cf[6]};
                        const int reg = (int)cf[7];
                        if (reg != 0 && pm != 0.0) {
                            const double ndn = nm[0] * dn[0] + nm[1] * dn[1] + nm[2] * dn[2];
                            const double edn = em[0] * dn[0] + em[1] * dn[1] + em[2] * dn[2];
                            for (int d = 0; d < 3; ++d) dx[d] += (dn[d] - ndn * nm[d] - edn * em[d]) / pm;
                        }
                    }
                }
            }
            for (int d = 0; d < 3; ++d) {
                G(S.gx)[3 * i + d] = dx[d] + (has_gstep ? gstep[3 * i + d] : 0.0);
                G(S.gv)[3 * i + d] = mi * z[d];
            }
            if (has_force)
                for (int d = 0; d < 3; ++d) {
                    G(S.dfext)[3 * i + d] += h * fs * z[d];
                    fz += G(S.fext)[3 * i + d] * z[d];
                }
        }
        if (has_force) {
            const double v = block_sum(fz, red);            // one fixed-order sum per step
            if (threadIdx.x == 0) G(S.dfscale)[n] = h * v;
        }
        for (int o = 0; o < S.n_obst; ++o) {
            const double v = block_sum(dmu_local[o], red);   // one fixed-order sum per step
            if (threadIdx.x == 0) G(S.dmu)[o] += v;
        }
        if (S.self_on) {
            const double v = block_sum(dmu_self, red);
            if (threadIdx.x == 0) G(S.dmu)[kMaxObstacles] += v;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        G(S.counters)[1] += iters_total;
        G(S.counters)[3] += noconv;
        G(S.counters)[4] += gm_total;
        G(S.counters)[5] += pert_total;
    }
    if constexpr (direct) publish_pos(S, kPosMask);      // releases the prefetch helpers
}

// ------------------------------------------------------------------ small helper kernels

// out[perm[i]] = in[i] (new -> caller order) or out[i] = in[perm[i]] (caller -> new), 3 per node
__global__ void k_permute3(const double *__restrict__ in, double *__restrict__ out, const int32_t *__restrict__ perm,
                           int m, int to_caller) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int o = perm[i];
    if (to_caller) {
        out[3 * o] = in[3 * i]; out[3 * o + 1] = in[3 * i + 1]; out[3 * o + 2] = in[3 * i + 2];
    } else {
        out[3 * i] = in[3 * o]; out[3 * i + 1] = in[3 * o + 1]; out[3 * i + 2] = in[3 * o + 2];
    }
}

__global__ void k_modes_to_caller(const uint8_t *__restrict__ in, uint8_t *__restrict__ out,
                                  const int32_t *__restrict__ perm, int m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) out[perm[i]] = in[i];
}

// dregion[r] = sum_c base_w[c] dw[c] over constraints of region r (one workgroup)
__global__ __launch_bounds__(kBlock) void k_region_grad(const double *__restrict__ dw, const double *__restrict__ base_w,
                                                        const int32_t *__restrict__ region, int nc, int nreg,
                                                        double *__restrict__ out) {
    __shared__ double red[kBlock / 64];
    for (int r = 0; r < nreg; ++r) {
        double acc = 0.0;
        for (int c = threadIdx.x; c < nc; c += (int)blockDim.x)
            if (region[c] == r) acc += base_w[c] * dw[c];
        acc = block_sum(acc, red);
        if (threadIdx.x == 0) out[r] = acc;
    }
}

// bending gradients: dw_bend[center] = dw[n_edges + b]
__global__ void k_scatter_bend(const double *__restrict__ dw, const int32_t *__restrict__ centers, int n_edges,
                               int n_bend, double *__restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < n_bend) out[centers[b]] = dw[n_edges + b];
}

__global__ void k_fill(double *p, double v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ launchers

template <bool MIXED, int FL>
static void fwd_one(const SimDev *d, int n, size_t lds, int helpers, hipStream_t st) {
    // helpers: handle h's solver at 8 (H+1) (h / 8) + h mod 8, its helpers 8, 16, .. above (same XCD)
    const int grid = helpers > 0 ? kXcds * (helpers + 1) * ((n + kXcds - 1) / kXcds) : n;
    hipLaunchKernelGGL((k_forward<MIXED, FL>), dim3(grid), dim3(kBlock), lds, st, d, n, helpers);
}
template <bool MIXED, int FL>
static void bwd_one(const SimDev *d, int n, size_t lds, int helpers, hipStream_t st) {
    // helpers (n == 1 only): workgroups kXcds, 2 kXcds, ... share the solver's XCD; the rest exit at once
    const int grid = helpers > 0 ? 1 + kXcds * helpers : n;
    hipLaunchKernelGGL((k_backward<MIXED, FL>), dim3(grid), dim3(kBlockAdj), lds, st, d, helpers);
}

#define DC_V16(f, M) f<M, 0>, f<M, 1>, f<M, 2>, f<M, 3>, f<M, 4>, f<M, 5>, f<M, 6>, f<M, 7>, \
    f<M, 8>, f<M, 9>, f<M, 10>, f<M, 11>, f<M, 12>, f<M, 13>, f<M, 14>, f<M, 15>

// mesh: a handle of the launch has a triangle-mesh obstacle (the kMeshObst variant)
hipError_t launch_forward(const SimDev *d_sims, int n, bool mixed, size_t lds, int flags, int helpers, bool mesh,
                          hipStream_t st) {
    using F = void (*)(const SimDev *, int, size_t, int, hipStream_t);
    static const F tab[2][16] = {{DC_V16(fwd_one, false)}, {DC_V16(fwd_one, true)}};
    tab[mixed ? 1 : 0][(flags & 7) | (mesh ? kMeshObst : 0)](d_sims, n, lds, helpers, st);
    return hipGetLastError();
}

hipError_t launch_backward(const SimDev *d_sims, int n, bool mixed, size_t lds, int flags, int helpers, bool mesh,
                           hipStream_t st) {
    if (helpers > 0 && n != 1) return hipErrorInvalidValue;
    using F = void (*)(const SimDev *, int, size_t, int, hipStream_t);
    static const F tab[2][16] = {{DC_V16(bwd_one, false)}, {DC_V16(bwd_one, true)}};
    tab[mixed ? 1 : 0][(flags & 7) | (mesh ? kMeshObst : 0)](d_sims, n, lds, helpers, st);
    return hipGetLastError();
}

// multi-workgroup forward of one handle (d: its descriptor), grid 8 W, lds
// bytes of dynamic LDS; lw: each workgroup solves its one subtree in LDS
hipError_t launch_forward_mw(const SimDev *d, int W, bool mixed, bool mesh, bool lw, size_t lds, int threads,
                             hipStream_t st) {
    if (W < 2 || W > kMwMax) return hipErrorInvalidValue;
    if (threads < 64 || threads > kBlock || threads % 64 != 0) return hipErrorInvalidValue;
    using F = void (*)(const SimDev *);
    static const F tab[2][2][2] = {{{k_forward_mw<false, false, false>, k_forward_mw<false, false, true>},
                                    {k_forward_mw<false, true, false>, k_forward_mw<false, true, true>}},
                                   {{k_forward_mw<true, false, false>, k_forward_mw<true, false, true>},
                                    {k_forward_mw<true, true, false>, k_forward_mw<true, true, true>}}};
    hipLaunchKernelGGL(tab[mixed][mesh][lw], dim3(kXcds * W), dim3(threads), lds, st, d);
    return hipGetLastError();
}

hipError_t configure_mw_lds(size_t bytes) {
    hipError_t e = hipSuccess, r;
    for (const void *f : {(const void *)k_forward_mw<false, false, false>, (const void *)k_forward_mw<false, false, true>,
                          (const void *)k_forward_mw<false, true, false>, (const void *)k_forward_mw<false, true, true>,
                          (const void *)k_forward_mw<true, false, false>, (const void *)k_forward_mw<true, false, true>,
                          (const void *)k_forward_mw<true, true, false>, (const void *)k_forward_mw<true, true, true>})
        if ((r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) e = r;
    return e;
}

// Allow the dynamic LDS the kernels may request (data resident in LDS).
template <bool MIXED, int FL>
static hipError_t set_fwd(size_t bytes) {
    return hipFuncSetAttribute((const void *)k_forward<MIXED, FL>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
template <bool MIXED, int FL>
static hipError_t set_bwd(size_t bytes) {
    return hipFuncSetAttribute((const void *)k_backward<MIXED, FL>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t configure_lds(size_t fwd_bytes, size_t bwd_bytes) {
    hipError_t e = hipSuccess, r;
#define DC_SETF(M, F) if ((r = set_fwd<M, F>(fwd_bytes)) != hipSuccess) e = r;
#define DC_SETB(M, F) if ((r = set_bwd<M, F>(bwd_bytes)) != hipSuccess) e = r;
#define DC_SET16(X, M) X(M, 0) X(M, 1) X(M, 2) X(M, 3) X(M, 4) X(M, 5) X(M, 6) X(M, 7) \
    X(M, 8) X(M, 9) X(M, 10) X(M, 11) X(M, 12) X(M, 13) X(M, 14) X(M, 15)
    DC_SET16(DC_SETF, false) DC_SET16(DC_SETF, true)
    DC_SET16(DC_SETB, false) DC_SET16(DC_SETB, true)
#undef DC_SET16
#undef DC_SETF
#undef DC_SETB
    return e;
}

// Largest static LDS over the kernel variants (reductions, GMRES workspace).
hipError_t kernel_static_lds(size_t *fwd, size_t *bwd) {
    hipFuncAttributes a;
    *fwd = 0;
    *bwd = 0;
    const void *fk[] = {(const void *)k_forward<false, 0>, (const void *)k_forward<false, 7>,
                        (const void *)k_forward<true, 0>, (const void *)k_forward<true, 7>,
                        (const void *)k_forward<false, 8>, (const void *)k_forward<true, 15>};
    const void *bk[] = {(const void *)k_backward<false, 0>, (const void *)k_backward<false, 3>,
                        (const void *)k_backward<true, 0>, (const void *)k_backward<true, 3>,
                        (const void *)k_backward<false, 4>, (const void *)k_backward<false, 7>,
                        (const void *)k_backward<true, 4>, (const void *)k_backward<true, 7>,
                        (const void *)k_backward<false, 8>, (const void *)k_backward<true, 15>};
    for (const void *f : fk) {
        hipError_t e = hipFuncGetAttributes(&a, f);
        if (e != hipSuccess) return e;
        *fwd = a.sharedSizeBytes > *fwd ? a.sharedSizeBytes : *fwd;
    }
    for (const void *f : bk) {
        hipError_t e = hipFuncGetAttributes(&a, f);
        if (e != hipSuccess) return e;
        *bwd = a.sharedSizeBytes > *bwd ? a.sharedSizeBytes : *bwd;
    }
    return hipSuccess;
}

hipError_t launch_adj_assemble(const SimDev *d_sims, const int32_t *work, int nblocks, hipStream_t st) {
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_assemble, dim3(nblocks), dim3(kFacBlock), 0, st, d_sims, work);
    return hipGetLastError();
}

// nmax: largest diagonal block of the launch's chunks (degrees of freedom, <= kGjMax)
hipError_t launch_adj_factor_level(const SimDev *d_sims, const int32_t *work, int nblocks, int nmax, hipStream_t st) {
    if (nblocks <= 0) return hipSuccess;
    if (nmax > kGjMax) return hipErrorInvalidValue;
    if (nmax <= 96) hipLaunchKernelGGL(k_adj_factor_level<6>, dim3(nblocks), dim3(kFacBlock), 0, st, d_sims, work);
    else hipLaunchKernelGGL(k_adj_factor_level<8>, dim3(nblocks), dim3(kFacBlock), 0, st, d_sims, work);
    return hipGetLastError();
}

hipError_t launch_permute3(const double *in, double *out, const int32_t *perm, int m, bool to_caller, hipStream_t st) {
    hipLaunchKernelGGL(k_permute3, dim3((m + 255) / 256), dim3(256), 0, st, in, out, perm, m, to_caller ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_modes(const uint8_t *in, uint8_t *out, const int32_t *perm, int m, hipStream_t st) {
    hipLaunchKernelGGL(k_modes_to_caller, dim3((m + 255) / 256), dim3(256), 0, st, in, out, perm, m);
    return hipGetLastError();
}

hipError_t launch_region_grad(const double *dw, const double *base_w, const int32_t *region, int nc, int nreg,
                              double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_region_grad, dim3(1), dim3(kBlock), 0, st, dw, base_w, region, nc, nreg, out);
    return hipGetLastError();
}

hipError_t launch_scatter_bend(const double *dw, const int32_t *centers, int n_edges, int n_bend, double *out,
                               hipStream_t st) {
    if (n_bend <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_bend, dim3((n_bend + 255) / 256), dim3(256), 0, st, dw, centers, n_edges, n_bend, out);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, double v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ allocation-free forward
// Work memory of sim_forward_noalloc: a file-scope device array, one per GPU
// (each device that loads the library holds its own copy until the process
// ends).  Host code never uses the array's name as an address: its device
// address is taken once per device with hipGetSymbolAddress and kept.  Every
// call on one GPU shares that GPU's array, so such calls must not overlap.
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

hipError_t noalloc_scratch(void **out) {
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

}  // namespace dc
