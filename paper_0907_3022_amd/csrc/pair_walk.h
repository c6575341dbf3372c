// Two Chebyshev orders per pass for brick-wall lattices: the walk of one
// wavefront over its strip and row chunk, shared by the single-system kernel
// (pair.hip) and the batched one (batch.hip).  The recursion is that of
// Sect. 2.2 of arXiv:0907.3022:
//   v_{k+1} = 2 H~ v_k - v_{k-1},   v_{k+2} = 2 H~ v_{k+1} - v_k,
//   acc += g_{k+1} v_{k+1} + g_{k+2} v_{k+2}
// (head variant: v_1 = H~ psi, v_2 = 2 H~ v_1 - psi,
//  acc = g_0 psi + g_1 v_1 + g_2 v_2, plus norm and energy sums).
//
// Lane l holds column x = 62*strip + l - 1, so lanes 0 and 63 are halo
// columns whose v_{k+1} the neighbouring lanes need for the second order.
// The wavefront walks down its rows keeping three rows of v_k and three of
// v_{k+1} in registers: vertical neighbours come from registers, horizontal
// ones from the adjacent lanes (cross-lane shuffles); only lanes 0 and 63
// load one extra v_k value per row.  A chunk of rows [ys, ye) computes
// v_{k+1} on rows ys-1 .. ye (one halo row each side, recomputed by the
// neighbouring chunk) and v_{k+2} on its own rows.  Outputs must go to
// buffers distinct from the inputs, since neighbouring wavefronts still read
// the inputs' halo rows.
#pragma once

#include <hip/hip_runtime.h>

#include "device_ops.h"
#include "pair.h"

namespace chebtd {

constexpr int kPairStrip = kPairStripCols;

namespace pairdev {

// Component-wise select by value.  A ternary between two double2 objects can
// make the compiler pick between their addresses, which sends them through
// scratch memory; selecting the scalars keeps everything in registers.
__device__ __forceinline__ double2 csel(bool c, double2 a, double2 b)
{
    return make_double2(c ? a.x : b.x, c ? a.y : b.y);
}

// Whole-wavefront shifts by one lane through DPP (a register move, no LDS
// round trip): from_left gives lane l the value of lane l-1 and lane 0 the
// value `edge`; from_right gives lane l the value of lane l+1 and lane 63
// `edge`.
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v, double edge)
{
    const long long b = __double_as_longlong(v), o = __double_as_longlong(edge);
    const int lo = __builtin_amdgcn_update_dpp((int)(o & 0xffffffff), (int)(b & 0xffffffff), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int kWaveShr1 = 0x138, kWaveShl1 = 0x130;
__device__ __forceinline__ double2 from_left(double2 v, double2 edge)
{
    return make_double2(dpp_shift<kWaveShr1>(v.x, edge.x), dpp_shift<kWaveShr1>(v.y, edge.y));
}
__device__ __forceinline__ double2 from_right(double2 v, double2 edge)
{
    return make_double2(dpp_shift<kWaveShl1>(v.x, edge.x), dpp_shift<kWaveShl1>(v.y, edge.y));
}
// the same shifts where the edge lane's result is not used (it reads 0)
template <int CTRL>
__device__ __forceinline__ double dpp_shift0(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double2 from_left0(double2 v)
{
    return make_double2(dpp_shift0<kWaveShr1>(v.x), dpp_shift0<kWaveShr1>(v.y));
}
__device__ __forceinline__ double2 from_right0(double2 v)
{
    return make_double2(dpp_shift0<kWaveShl1>(v.x), dpp_shift0<kWaveShl1>(v.y));
}

// Operands of one row loaded one iteration ahead: v_k of the row below,
// and v_{k-1}, the on-site term, the outside v_k value (strip-edge lanes) and
// acc of the row itself.
struct Prefetch {
    double2 a, km1, ext, acc;
    double e;
};

}  // namespace pairdev

// The wavefront's share: strip `strip` (62 columns), rows
// [chunk*op.rows, min((chunk+1)*op.rows, W)).  nrm/en accumulate the head's
// norm and energy terms of the lane's own sites.  Without ACC only the two
// new vectors are written (the adjoint's recomputation of the forward
// vectors): acc, the weights, ckpt and the sums are not touched.
template <int EDGE, bool HEAD, bool ACC = true>
__device__ __forceinline__ void pair_walk(const OpPair &op, int32_t strip, int32_t chunk,
                                          const double2 *__restrict__ vkm1, const double2 *__restrict__ vk,
                                          double2 *__restrict__ out1, double2 *__restrict__ out2,
                                          double2 *__restrict__ acc, double2 g0, double2 g1, double2 g2,
                                          double2 *__restrict__ ckpt, double &nrm, double &en)
{
    using namespace pairdev;
    const int lane = threadIdx.x & 63;
    const int32_t W = op.W, L = op.L;
    const int32_t x = strip * kPairStrip + lane - 1;
    const bool colok = x >= 0 && x < L;
    const bool own = colok && lane >= 1 && lane <= kPairStrip;
    const double2 zero = make_double2(0.0, 0.0);
    const int32_t ys = chunk * op.rows;
    const int32_t ye = min(ys + op.rows, W);
    // Loads are unconditional, from a clamped index, and return the raw
    // value; where a zero is needed outside the lattice it is selected
    // when the value is used, one row later.  (A conditional load of
    // memory or a local zero becomes a flat load of a selected pointer,
    // and selecting right after the load would make every iteration wait
    // for the prefetch it has just issued.)
    auto okr = [&](int32_t r) -> bool { return colok && r >= 0 && r < W; };
    auto ld = [&](const double2 *v, int32_t r) -> double2 {
        return ldg(v, okr(r) ? (int64_t)r * L + x : 0);
    };
    auto ld_on = [&](int32_t r) -> double { return ldg(op.onsite, okr(r) ? (int64_t)r * L + x : 0); };
    // lanes 0 and 63 also need the v_k value just outside the strip
    const int32_t xe = lane == 0 ? x - 1 : x + 1;
    const bool ext_lane = (lane == 0 || lane == 63) && xe >= 0 && xe < L;
    auto ok_ext = [&](int32_t r) -> bool { return ext_lane && r >= 0 && r < W; };
    auto ld_ext = [&](int32_t r) -> double2 { return ldg(vk, ok_ext(r) ? (int64_t)r * L + xe : 0); };
    auto st = [&](double2 *v, int32_t r, double2 val) { stg(v, (int64_t)r * L + x, val); };
    // operands of row r (v_k row r+1, v_{k-1}, on-site and outside value of
    // row r, acc of row r-1) are loaded one iteration ahead; v_{k-1}, the
    // on-site term and acc are only used where they are in range
    double2 a_m1 = csel(okr(ys - 2), ld(vk, ys - 2), zero);  // v_k rows r-1, r
    double2 a_0 = csel(okr(ys - 1), ld(vk, ys - 1), zero);
    // Two sets of prefetch registers, used alternately: the loads issued
    // for the next row are never copied (a copy would wait for them).
    Prefetch p0, p1;
    p0.a = ld(vk, ys);
    p0.km1 = HEAD ? zero : ld(vkm1, ys - 1);
    p0.e = ld_on(ys - 1);
    p0.ext = ld_ext(ys - 1);
    p0.acc = zero;
    double2 b_m2 = zero, b_m1 = zero;  // v_{k+1} rows r-2, r-1
    double e_m1 = 0.0;                 // on-site term, row r-1
    // one row: prefetch row r+1 into nx, compute from cur
    auto row_step = [&](int32_t r, const Prefetch &cur, Prefetch &nx) {
        nx.a = ld(vk, r + 2);
        nx.km1 = HEAD ? zero : ld(vkm1, r + 1);
        nx.e = ld_on(r + 1);
        nx.ext = ld_ext(r + 1);
        if (ACC && !HEAD) {
            const bool ok = own && r >= ys && r < ye;
            nx.acc = ldg(acc, ok ? (int64_t)r * L + x : 0);
        }
        const double2 a_p1 = csel(okr(r + 1), cur.a, zero);
        const double2 ext = csel(ok_ext(r), cur.ext, zero);
        const double e_0 = cur.e;
        const bool rowok = r >= 0 && r < W;
        // ---- first order at row r: v_{k+1} = 2 H~ v_k - v_{k-1} ----
        const double2 left = from_left(a_0, ext), right = from_right(a_0, ext);
        const bool even_r = ((x + r) & 1) == 0;
        double2 s;
        if (EDGE == CHEBTD_ZIGZAG)
            s = cadd(cadd(left, right), csel(even_r, a_p1, a_m1));
        else
            s = cadd(cadd(a_m1, a_p1), csel(even_r, right, left));
        const double d0 = op.s2 * (e_0 + op.dshift);
        const double2 h = make_double2(fma(d0, a_0.x, op.off2 * s.x), fma(d0, a_0.y, op.off2 * s.y));
        double2 b_0 = HEAD ? cscale(0.5, h) : csub(h, cur.km1);
        b_0 = csel(colok && rowok, b_0, zero);
        if (own && r >= ys && r < ye) st(out1, r, b_0);
        // ---- second order at row q = r-1: v_{k+2} = 2 H~ v_{k+1} - v_k ----
        if (r - 1 >= ys) {
            const int32_t q = r - 1;
            // lanes 0 and 63 get no second order: their edge value is unused
            const double2 l2 = from_left0(b_m1), r2 = from_right0(b_m1);
            const bool even_q = ((x + q) & 1) == 0;
            double2 s2;
            if (EDGE == CHEBTD_ZIGZAG)
                s2 = cadd(cadd(l2, r2), csel(even_q, b_0, b_m2));
            else
                s2 = cadd(cadd(b_m2, b_0), csel(even_q, r2, l2));
            const double d1 = op.s2 * (e_m1 + op.dshift);
            const double2 h2 = make_double2(fma(d1, b_m1.x, op.off2 * s2.x), fma(d1, b_m1.y, op.off2 * s2.y));
            const double2 c = csub(h2, a_m1);
            if (own) st(out2, q, c);
            if (ACC && own) {
                double2 a;
                if (HEAD) {
                    a = cfma(g0, a_m1, zero);
                    if (ckpt) st(ckpt, q, a_m1);
                    nrm += a_m1.x * a_m1.x + a_m1.y * a_m1.y;
                    en += a_m1.x * b_m1.x + a_m1.y * b_m1.y;
                } else {
                    a = cur.acc;  // acc of row q, loaded with the previous row
                }
                a = cfma(g1, b_m1, a);
                st(acc, q, cfma(g2, c, a));
            }
        }
        a_m1 = a_0;
        a_0 = a_p1;
        b_m2 = b_m1;
        b_m1 = b_0;
        e_m1 = e_0;
    };
    int32_t r = ys - 1;
    for (; r + 1 <= ye; r += 2) {
        row_step(r, p0, p1);
        row_step(r + 1, p1, p0);
    }
    if (r <= ye) row_step(r, p0, p1);
}

}  // namespace chebtd
