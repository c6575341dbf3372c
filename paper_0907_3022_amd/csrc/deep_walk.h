// D Chebyshev orders per pass for brick-wall lattices (the honeycomb ribbons
// of eq. (model), the 1D chain as a ribbon of one row): the Sect. 2.2
// recursion of arXiv:0907.3022 carried D levels deep inside one walk,
//   v_{k+j} = 2 H~ v_{k+j-1} - v_{k+j-2},   j = 1..D,
//   acc += sum_j g_{k+j} v_{k+j},
// reading v_{k-1}, v_k, the on-site term and acc once and writing only
// v_{k+D-1}, v_{k+D} and acc: 104 B per site for all D orders.  (The head
// variant starts a step: v_1 = H~ psi, acc = g_0 psi + sum_j g_j v_j, with
// the norm and energy sums.)
//
// The walk generalises the two-level one of pair_walk.h.  At iteration r
// level j computes row r - (j-1) from level j-1's window of three rows and
// level j-2's value at the same row, so every level keeps rows
// q-2 .. q of its own values in registers.  Horizontally each level past the
// first loses one valid lane per side: a wavefront owns the 66 - 2D columns
// on lanes D-1 .. 64-D.  Vertically level j is needed on rows
// ys - (D-j) .. ye - 1 + (D-j) of the chunk [ys, ye); the neighbouring
// chunks recompute those halo rows.  acc of a row collects its D terms over
// D iterations in a ring of partial sums.
#pragma once

#include <hip/hip_runtime.h>

#include "device_ops.h"
#include "pair.h"
#include "pair_walk.h"

namespace chebtd {

template <int D>
struct DeepWeights {
    double2 g[D + 1];  // g_{k}, g_{k+1} .. g_{k+D} (g_k only used by the head: gamma_0)
};

constexpr int deep_strip(int D) { return 66 - 2 * D; }

namespace deepdev {

struct Prefetch {
    double2 a, km1, ext, acc;
    double e;
};

}  // namespace deepdev

template <int EDGE, int D, bool HEAD>
__device__ __forceinline__ void deep_walk(const OpPair &op, int32_t strip, int32_t chunk,
                                          const double2 *__restrict__ vkm1, const double2 *__restrict__ vk,
                                          double2 *__restrict__ out1, double2 *__restrict__ out2,
                                          double2 *__restrict__ acc, const DeepWeights<D> &gw,
                                          double2 *__restrict__ ckpt, double &nrm, double &en)
{
    static_assert(D >= 2 && D <= 6, "depth");
    using namespace pairdev;
    using deepdev::Prefetch;
    constexpr int S = deep_strip(D);
    const int lane = threadIdx.x & 63;
    const int32_t W = op.W, L = op.L;
    const int32_t x = strip * S + lane - (D - 1);
    const bool colok = x >= 0 && x < L;
    const bool own = colok && lane >= D - 1 && lane <= 64 - D;
    const double2 zero = make_double2(0.0, 0.0);
    const int32_t ys = chunk * op.rows;
    const int32_t ye = min(ys + op.rows, W);
    // unconditional loads from clamped indices; zeros outside the lattice
    // are selected when a value is used (see pair_walk.h)
    auto okr = [&](int32_t r) -> bool { return colok && r >= 0 && r < W; };
    auto ld = [&](const double2 *v, int32_t r) -> double2 { return ldg(v, okr(r) ? (int64_t)r * L + x : 0); };
    auto ld_on = [&](int32_t r) -> double { return ldg(op.onsite, okr(r) ? (int64_t)r * L + x : 0); };
    const int32_t xe = lane == 0 ? x - 1 : x + 1;
    const bool ext_lane = (lane == 0 || lane == 63) && xe >= 0 && xe < L;
    auto ok_ext = [&](int32_t r) -> bool { return ext_lane && r >= 0 && r < W; };
    auto ld_ext = [&](int32_t r) -> double2 { return ldg(vk, ok_ext(r) ? (int64_t)r * L + xe : 0); };
    auto ld_acc = [&](int32_t r) -> double2 {
        const bool ok = own && r >= ys && r < ye;
        return ldg(acc, ok ? (int64_t)r * L + x : 0);
    };
    auto st = [&](double2 *v, int32_t r, double2 val) { stg(v, (int64_t)r * L + x, val); };

    const int32_t r0 = ys - (D - 1);   // first iteration: level 1 at its first needed row
    const int32_t r1 = ye + (D - 2);   // last iteration: level D at row ye - 1
    // level 0 (v_k) rows r-1, r; level j >= 1 rows q_j-2, q_j-1, q_j
    double2 a_m1 = csel(okr(r0 - 1), ld(vk, r0 - 1), zero);
    double2 a_0 = csel(okr(r0), ld(vk, r0), zero);
    double2 lv[D + 1][3];
#pragma unroll
    for (int j = 0; j <= D; ++j) lv[j][0] = lv[j][1] = lv[j][2] = zero;
    double e[D];  // on-site term of rows r, r-1, .., r-D+1
#pragma unroll
    for (int j = 0; j < D; ++j) e[j] = 0.0;
    double2 P[D];  // partial acc of rows r, r-1, .., r-D+1
#pragma unroll
    for (int j = 0; j < D; ++j) P[j] = zero;
    Prefetch p0, p1;
    p0.a = ld(vk, r0 + 1);
    p0.km1 = HEAD ? zero : ld(vkm1, r0);
    p0.e = ld_on(r0);
    p0.ext = ld_ext(r0);
    p0.acc = HEAD ? zero : ld_acc(r0);

    // stencil: 2 H~ of level `lo` at row q from its window (m, c, p = rows
    // q-1, q, q+1) with the horizontal neighbours of c
    auto stencil = [&](double2 m, double2 c, double2 p, double2 left, double2 right, int32_t q, double eq) {
        const bool even = ((x + q) & 1) == 0;
        double2 sum;
        if (EDGE == CHEBTD_ZIGZAG)
            sum = cadd(cadd(left, right), csel(even, p, m));
        else
            sum = cadd(cadd(m, p), csel(even, right, left));
        const double d = op.s2 * (eq + op.dshift);
        return make_double2(fma(d, c.x, op.off2 * sum.x), fma(d, c.y, op.off2 * sum.y));
    };

    auto row_step = [&](int32_t r, const Prefetch &cur, Prefetch &nx) {
        nx.a = ld(vk, r + 2);
        nx.km1 = HEAD ? zero : ld(vkm1, r + 1);
        nx.e = ld_on(r + 1);
        nx.ext = ld_ext(r + 1);
        if (!HEAD) nx.acc = ld_acc(r + 1);
        const double2 a_p1 = csel(okr(r + 1), cur.a, zero);
        const double2 ext = csel(ok_ext(r), cur.ext, zero);
        // on-site ring: e[j] = row r - j
#pragma unroll
        for (int j = D - 1; j > 0; --j) e[j] = e[j - 1];
        e[0] = cur.e;
        // level 0 window for this iteration: rows r-1, r, r+1
        lv[0][0] = a_m1;
        lv[0][1] = a_0;
        lv[0][2] = a_p1;
#pragma unroll
        for (int j = 1; j <= D; ++j) {
            const int32_t q = r - (j - 1);
            double2 val = zero;
            // level j is needed on rows ys - (D-j) .. ye - 1 + (D-j), and
            // is zero outside the lattice's rows
            if (q >= max(ys - (D - j), 0) && q <= min(ye - 1 + (D - j), W - 1)) {
                const double2 c = lv[j - 1][1];
                double2 left, right;
                if (j == 1) {
                    left = from_left(c, ext);
                    right = from_right(c, ext);
                } else {
                    left = from_left0(c);
                    right = from_right0(c);
                }
                const double2 h = stencil(lv[j - 1][0], c, lv[j - 1][2], left, right, q, e[j - 1]);
                if (j == 1)
                    val = HEAD ? cscale(0.5, h) : csub(h, cur.km1);
                else
                    val = csub(h, j == 2 ? lv[0][0] : lv[j - 2][0]);
                val = csel(colok, val, zero);
            }
            lv[j][0] = lv[j][1];
            lv[j][1] = lv[j][2];
            lv[j][2] = val;
            // partial acc of row q
            if (j == 1) {
                P[0] = cfma(gw.g[1], val, HEAD ? cfma(gw.g[0], a_0, zero) : cur.acc);
                if (HEAD && own && r >= ys && r < ye) {
                    if (ckpt) st(ckpt, r, a_0);
                    nrm += a_0.x * a_0.x + a_0.y * a_0.y;
                    en += a_0.x * val.x + a_0.y * val.y;
                }
            } else {
                P[j - 1] = cfma(gw.g[j], val, P[j - 1]);
            }
            if (own && q >= ys && q < ye) {
                if (j == D - 1) st(out1, q, val);
                if (j == D) {
                    st(out2, q, val);
                    st(acc, q, P[D - 1]);
                }
            }
        }
        // partial-acc ring: P[j] = row r - j for the next iteration
#pragma unroll
        for (int j = D - 1; j > 0; --j) P[j] = P[j - 1];
        a_m1 = a_0;
        a_0 = a_p1;
    };
    int32_t r = r0;
    for (; r + 1 <= r1; r += 2) {
        row_step(r, p0, p1);
        row_step(r + 1, p1, p0);
    }
    if (r <= r1) row_step(r, p0, p1);
}

}  // namespace chebtd
