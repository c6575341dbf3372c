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
// level j-2's value at the same row, so levels 0 .. D-1 keep three rows each
// in registers.  Horizontally each level past the first loses one valid lane
// per side: a wavefront owns the 66 - 2D columns on lanes D-1 .. 64-D.
// Vertically level j is needed on rows ys - (D-j) .. ye - 1 + (D-j) of the
// chunk [ys, ye); the neighbouring chunks recompute those halo rows.  acc of
// a row collects its D terms over D iterations in a ring of partial sums.
//
// Register rings without moves: the row a level writes at iteration i goes
// to window slot i mod 3, the partial sum and the diagonal term of row r - t
// sit in slot (i - t) mod deep_ring(D), and the operands loaded kDeepAhead
// iterations ahead rotate through kDeepAhead + 1 sets.  The loop body is
// unrolled over a common multiple of the ring sizes, so every slot index is
// a constant and no value is copied between registers.
//
// The same walk serves four uses (MODE): the propagation step above; the
// recomputation of a step's Chebyshev vectors for the adjoint, each level
// stored to its own vector and nothing accumulated; the adjoint's reverse
// recursion, level j forming
//   u_{k-j+1} = conj(g_{k-j+1}) gbar + 2 H~ u_{k-j+2} - u_{k-j+3}
// from u_{k+1} (level 0) and u_{k+2}, while dL/dV of a row collects
// (2/a) Re[conj(u_{k-j+2}) v_{k-j+1}] from every level in a ring like acc's,
// the forward vectors v read from memory; and that reverse recursion with
// the forward vectors regenerated beside it, from v_{k+1} and v_k, by the
// same three-term recursion run downwards,
//   v_{k-j} = 2 H~ v_{k-j+1} - v_{k-j+2},
// a second set of D windows in the same walk (exact in exact arithmetic;
// with the rescaled spectrum inside [-1, 1] a rounding error grows no faster
// run downwards than upwards, bounded by the Chebyshev polynomials of the
// second kind).  The last level of such a pass may be the recursion's
// level 0, u_0 = conj(g_0) gbar + H~ u_1 - u_2 with dL/dV share
// (1/a) Re[conj(u_1) v_0]: hD and gfD carry its halved factors.
//
// Memory goes through buffer loads and stores whose 32-bit offsets wrap:
// rows above or below the lattice, columns outside it and lanes that own no
// column get offsets at or past the buffer's size, which the hardware's
// range check turns into zeros (loads) or dropped writes (stores), so the
// walk selects nothing per row.  deep_offsets_fit states the size limit.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_ops.h"
#include "pair.h"
#include "pair_walk.h"

namespace chebtd {

template <int D>
struct DeepWeights {
    double2 g[D + 1];  // g_{k}, g_{k+1} .. g_{k+D} (g_k only used by the head: gamma_0)
};

constexpr int kDeepProp = 0;  // propagation: acc += sum_j g_{k+j} v_{k+j}
constexpr int kDeepAll = 1;   // recomputation: level j stored to all[j-1]
constexpr int kDeepAdj = 2;   // adjoint levels and dL/dV
constexpr int kDeepRev = 3;   // adjoint levels, dL/dV and the forward vectors run downwards

// Operands of one pass.  vkm1, vk: the two vectors entering level 1 (the
// adjoint's u_{k+2}, u_{k+1}; vkm1 may be null for the head, or for the
// adjoint's first pass, where u_{k+2} = 0); out1, out2: levels D-1 and D.
template <int D>
struct DeepArgs {
    const double2 *vkm1, *vk;
    double2 *out1, *out2;
    double2 *acc;            // propagation: read (not by the head) and written
    double2 *ckpt;           // propagation head: a copy of psi, or null
    double2 *all[D];         // recomputation: level j's vector
    const double2 *gbar;     // adjoint: dL/dpsi* of the step's result
    double *grad;            // adjoint: dL/dV, read and written
    const double2 *fwd;      // adjoint: v_{k-D+1}; level j's v_{k-j+1} lies (D-j) n after it
    double gf;               // adjoint: 2/a
    const double2 *rv1, *rv0;  // downwards: v_{k+1}, v_k
    double2 *rout1, *rout2;    // downwards: v_{k-D+1}, v_{k-D} (null: not stored)
    double hD;               // downwards: 1, or 1/2 when level D is the recursion's level 0
    double gfD;              // downwards: level D's dL/dV factor, 2/a or 1/a
    DeepWeights<D> w;        // propagation g_k .. g_{k+D}; adjoint conj(g_{k-j+1}) in w.g[j]
};

constexpr int deep_strip(int D) { return deep_strip_cols(D); }
constexpr int deep_gcd(int a, int b) { return b == 0 ? a : deep_gcd(b, a % b); }
constexpr int deep_lcm(int a, int b) { return a / deep_gcd(a, b) * b; }
// Iterations between issuing a row's loads and using them.  A wavefront
// walks its rows one after another, so the loads of the next row alone
// cannot cover the memory latency when few wavefronts share a SIMD.
constexpr int kDeepAhead = 1;
// Slots of the partial-sum and diagonal rings: at least D, and a divisor of
// 6 so that the unrolled body stays 6 iterations long for every depth.
constexpr int deep_ring(int D) { return 6 % D == 0 ? D : 6; }
// Propagation passes walk odd chunks upwards, so that both chunks next to a
// chunk boundary read the rows around it at the same time (both at the start
// of their walks or both at the end), and number wavefronts chunk-fastest
// within a strip, so that neighbouring chunks run on the same L2 and the
// second read of a boundary row hits it.  Measured on MI355X for five-order
// passes: 21.7 -> 20.4 us at 128x8192, 374 -> 366 us at 512x32768,
// 1478 -> 1426 us at 1024x65536 (the numbering alone was 3-5% slower).  A
// site's arithmetic is the same either way.
constexpr bool kDeepAlternate = true;
constexpr bool kDeepChunkFast = true;
// iterations per unrolled loop body: a multiple of kDeepAhead + 1
// (prefetch sets), 3 (row windows) and the ring size
constexpr int deep_unroll(int D) { return deep_lcm(deep_lcm(kDeepAhead + 1, 3), deep_ring(D)); }
// Iterations a walk of `rows` rows runs: whole unrolled bodies covering the
// rows + 2 (D - 1) it needs.  Chunk heights with rows + 2 (D - 1) a multiple
// of the body waste none.
constexpr int deep_iterations(int D, int rows)
{
    return (rows + 2 * (D - 1) + deep_unroll(D) - 1) / deep_unroll(D) * deep_unroll(D);
}

namespace deepdev {

using Rsrc = __amdgpu_buffer_rsrc_t;
// word 3 of the buffer descriptor for gfx9-family parts: 32-bit data format,
// raw (unswizzled) addressing
constexpr int kRsrcWord3 = 0x00020000;
constexpr uint32_t kOut = 0x80000000u;  // offset bias of out-of-lattice lanes

__device__ __forceinline__ Rsrc rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, kRsrcWord3);
}
// voff: the lane's offset; soff: a wave-uniform offset added to it
__device__ __forceinline__ double2 bload2(Rsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ double bload1(Rsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
// CPOL: the store's cache policy bits, 0 or kStreamStore
constexpr int kStreamStore = 2;  // non-temporal (streaming) on gfx950
template <int CPOL = 0>
__device__ __forceinline__ void bstore2(Rsrc r, uint32_t voff, uint32_t soff, double2 v)
{
    using V4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V4, v), r, (int)voff, (int)soff, CPOL);
}
__device__ __forceinline__ void bstore1(Rsrc r, uint32_t voff, uint32_t soff, double v)
{
    using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, (int)voff, (int)soff, 0);
}

// Operands of row rn loaded ahead: v_k of row rn+1 (the next level-0 row),
// and v_{k-1}, the on-site term, the outside value and acc (adjoint: gbar
// and dL/dV) of row rn; run downwards, the same three for the forward
// vectors (va, vkm1, vext).
struct DeepPrefetch {
    double2 a, km1, ext, acc;
    double2 va, vkm1, vext;
    double e, gr;
};

// f(integral_constant<PH>) for PH = 0 .. U-1
template <int PH, int U, typename F>
__device__ __forceinline__ void phases(F &f)
{
    if constexpr (PH < U) {
        f(std::integral_constant<int, PH>{});
        phases<PH + 1, U>(f);
    }
}

}  // namespace deepdev

// The wavefront's share: strip `strip` (66 - 2D columns), rows
// [chunk*op.rows, min((chunk+1)*op.rows, W)).  BORDER: the strip has lanes
// outside the lattice's columns, or the chunk's halo reaches past its first
// or last row; values outside the lattice must then stay zero, so each level
// is limited to its rows and masked to the lattice's columns.  Elsewhere a
// level also computes the rows before its first needed one; those only feed
// other such rows and are never stored.
// NT: the pass's vector stores stream past the caches (lattices far larger
// than the last-level cache: measured on MI355X, five-order passes at
// 512x32768 ran 366 -> 354 us; at 128x8192, whose vectors the next pass reads
// from that cache, 20.3 -> 29.2 us, so smaller lattices store normally)
template <int EDGE, int D, bool HEAD, bool BORDER, int MODE, bool UP = false, bool NT = false>
__device__ __forceinline__ void deep_walk(const OpPair &op, int32_t strip, int32_t chunk, const DeepArgs<D> &A,
                                          double &nrm, double &en)
{
    static_assert(D >= 2 && D <= 6, "depth");
    static_assert(!UP || MODE == kDeepProp, "only propagation walks upwards");
    constexpr int32_t dir = UP ? -1 : 1;  // rows walked downwards (+1) or upwards
    static_assert(MODE == kDeepProp || !HEAD || MODE == kDeepAll, "the adjoint has no head pass");
    constexpr bool PROP = MODE == kDeepProp, ALL = MODE == kDeepAll, REV = MODE == kDeepRev;
    constexpr bool ADJ = MODE == kDeepAdj || REV;  // the adjoint recursion, either way
    const DeepWeights<D> &gw = A.w;
    using namespace pairdev;
    using namespace deepdev;
    constexpr int S = deep_strip(D);
    constexpr int U = deep_unroll(D);
    const int lane = threadIdx.x & 63;
    const int32_t W = op.W, L = op.L;
    const int32_t x = strip * S + lane - (D - 1);
    const bool colok = x >= 0 && x < L;
    const bool own = colok && lane >= D - 1 && lane <= 64 - D;
    const double2 zero = make_double2(0.0, 0.0);
    const int32_t ys = chunk * op.rows;
    const int32_t nrows = min(op.rows, W - ys);  // rows of the chunk

    const uint32_t nb16 = (uint32_t)W * (uint32_t)L * 16u;
    // A missing buffer gets a descriptor of size 0: its loads read zeros and
    // its stores are dropped.
    auto rsrc_or_0 = [&](const void *p, uint32_t bytes) { return rsrc(p ? p : A.vk, p ? bytes : 0u); };
    const Rsrc rk = rsrc(A.vk, nb16), ron = rsrc(op.onsite, nb16 / 2);
    const Rsrc rkm1 = rsrc_or_0(HEAD ? nullptr : A.vkm1, nb16);
    const Rsrc ro1 = rsrc_or_0(ALL ? nullptr : A.out1, nb16), ro2 = rsrc_or_0(ALL ? nullptr : A.out2, nb16);
    const Rsrc racc = rsrc_or_0(PROP ? A.acc : ADJ ? A.gbar : nullptr, nb16);
    const Rsrc rck = rsrc_or_0(PROP && HEAD ? A.ckpt : nullptr, nb16);
    const Rsrc rgr = rsrc_or_0(ADJ ? A.grad : nullptr, nb16 / 2);
    // the adjoint's D forward vectors, n apart (D n 16 B <= 2^30, so the
    // out-of-range bias never wraps into them)
    const Rsrc rfw = rsrc_or_0(ADJ && !REV ? A.fwd : nullptr, ADJ && !REV ? (uint32_t)D * nb16 : 0u);
    // run downwards: the two forward vectors entering the pass and the two it leaves
    const Rsrc rv1 = rsrc_or_0(REV ? A.rv1 : nullptr, nb16), rv0 = rsrc_or_0(REV ? A.rv0 : nullptr, nb16);
    const Rsrc rvo1 = rsrc_or_0(REV ? A.rout1 : nullptr, nb16), rvo2 = rsrc_or_0(REV ? A.rout2 : nullptr, nb16);
    // column part of each offset: loads (lattice columns), stores (own
    // columns), the outside value (lanes 0 and 63); kOut elsewhere
    const uint32_t c16 = colok ? (uint32_t)x * 16u : kOut;
    const uint32_t c8 = colok ? (uint32_t)x * 8u : kOut;
    const uint32_t s16 = own ? (uint32_t)x * 16u : kOut;
    // The outside value of lanes 0 and 63 (columns x-1, x+1) enters the
    // stencil sum as one more term, zero on every other lane.  On armchair
    // edges a lane reads it only on rows where its horizontal neighbour is on
    // that side (lane 0 on odd x+q, lane 63 on even), so it is loaded there only.
    const int32_t xe = lane == 0 ? x - 1 : x + 1;
    const uint32_t e16 = ((lane == 0 || lane == 63) && xe >= 0 && xe < L) ? (uint32_t)xe * 16u : kOut;
    const int32_t epar = lane == 0 ? 1 : 0;
    auto ext_off = [&](int32_t q) -> uint32_t {
        if (EDGE == CHEBTD_ZIGZAG) return e16;
        return ((x + q) & 1) == epar ? e16 : kOut;
    };
    const uint32_t row16 = (uint32_t)L * 16u, row8 = (uint32_t)L * 8u;
    // Row part of an offset, wrapping for rows above the lattice.  On the
    // border it joins the lane's part, so that the range check sees rows
    // outside the lattice; inside, every row exists and it rides in the
    // instruction's scalar offset instead.
    auto ld2 = [&](Rsrc rs, uint32_t lanepart, int32_t row) -> double2 {
        const uint32_t ro = (uint32_t)row * row16;
        return BORDER ? bload2(rs, ro + lanepart, 0) : bload2(rs, lanepart, ro);
    };
    auto ld1 = [&](Rsrc rs, uint32_t lanepart, int32_t row) -> double {
        const uint32_t ro = (uint32_t)row * row8;
        return BORDER ? bload1(rs, ro + lanepart, 0) : bload1(rs, lanepart, ro);
    };
    // Store to the own columns of `row` if `ok`; otherwise the store is
    // issued anyway, from out-of-range lanes, and dropped (a branch here
    // would make every later wait drain all loads in flight).  The whole
    // offset goes in the lane's register and the scalar offset is 0: the
    // compiler then keeps the store's data registers unwritten for the wait
    // state that 128-bit stores need, which it assumes unnecessary when the
    // scalar offset is a register.  With that form, data written right after
    // the store intermittently reached memory in place of the stored values.
    auto st2 = [&](Rsrc rs, int32_t row, double2 v, bool ok) {
        const uint32_t ro = (uint32_t)row * row16;
        bstore2<NT ? kStreamStore : 0>(rs, ro + (ok ? s16 : kOut), 0, v);
    };
    const uint32_t s8 = own ? (uint32_t)x * 8u : kOut;
    auto st1 = [&](Rsrc rs, int32_t row, double v, bool ok) {
        const uint32_t ro = (uint32_t)row * row8;
        bstore1(rs, ro + (ok ? s8 : kOut), 0, v);
    };

    // iteration i: level j at row r0 + dir (i - (j-1))
    const int32_t r0 = UP ? ys + nrows - 1 + (D - 1) : ys - (D - 1);
    // windows of levels 0 .. D-1 (three rows each); partial sums and
    // diagonal terms 2 (eps - b)/a of the last RS rows
    constexpr int RS = deep_ring(D);
    double2 lv[D][3];
    double2 vl[REV ? D : 1][3];  // downwards: the forward vectors' windows
    double2 P[RS];   // propagation: partial acc; adjoint: gbar of the row
    double G[RS];    // adjoint: partial dL/dV
    double dd[RS];
#pragma unroll
    for (int j = 0; j < D; ++j) lv[j][0] = lv[j][1] = lv[j][2] = zero;
#pragma unroll
    for (int j = 0; j < (REV ? D : 1); ++j) vl[j][0] = vl[j][1] = vl[j][2] = zero;
#pragma unroll
    for (int j = 0; j < RS; ++j) {
        P[j] = zero;
        G[j] = 0.0;
        dd[j] = 0.0;
    }
    // iteration 0 reads level-0 rows r0-1 (slot 1) and r0 (slot 2)
    lv[0][1] = ld2(rk, c16, r0 - dir);
    lv[0][2] = ld2(rk, c16, r0);
    if (REV) {
        vl[0][1] = ld2(rv0, c16, r0 - dir);
        vl[0][2] = ld2(rv0, c16, r0);
    }
    // operands of iteration n (pair_walk.h's set: v_k of the row below, and
    // v_{k-1}, on-site term, outside value and acc of row r0 + n)
    constexpr int K = kDeepAhead + 1;
    DeepPrefetch pf[K];
    auto issue = [&](DeepPrefetch &nx, int32_t n) {
        const int32_t rn = r0 + dir * n;
        nx.a = ld2(rk, c16, rn + dir);
        if (!HEAD) nx.km1 = ld2(rkm1, c16, rn);
        nx.e = ld1(ron, c8, rn);
        nx.ext = ld2(rk, ext_off(rn), rn);
        // acc and dL/dV only where they are stored again (other rows' sums
        // are discarded); the adjoint's gbar on every row a level computes
        const int32_t rel = rn - ys;
        const bool ok = rel >= 0 && rel < nrows;
        if (PROP && !HEAD) nx.acc = ld2(racc, ok ? s16 : kOut, rn);
        if (ADJ) {
            nx.acc = ld2(racc, c16, rn);
            nx.gr = ld1(rgr, ok ? s8 : kOut, rn);
        }
        if (REV) {
            nx.va = ld2(rv0, c16, rn + dir);
            nx.vkm1 = ld2(rv1, c16, rn);
            nx.vext = ld2(rv0, ext_off(rn), rn);
        }
    };
#pragma unroll
    for (int k = 0; k < K; ++k) {
        pf[k].km1 = pf[k].acc = pf[k].va = pf[k].vkm1 = pf[k].vext = zero;
        pf[k].gr = 0.0;
        if (k < K - 1) issue(pf[k], k);
    }

    auto stencil_sum = [&](double2 m, double2 p, double2 left, double2 right, int32_t q) {
        const bool even = ((x + q) & 1) == 0;
        if (EDGE == CHEBTD_ZIGZAG) return cadd(cadd(left, right), csel(even, p, m));
        return cadd(cadd(m, p), csel(even, right, left));
    };

    int32_t base = 0;  // first iteration of the unrolled body
    auto step = [&](auto phc) {
        constexpr int ph = decltype(phc)::value;
        constexpr int sl0 = ph % 3, sl1 = (ph + 2) % 3, sl2 = (ph + 1) % 3;  // iterations i, i-1, i-2
        DeepPrefetch &cur = pf[ph % K];
        const int32_t i = base + ph;
        const int32_t rr = r0 + dir * i;
        // operands kDeepAhead iterations on, into the set freed last iteration;
        // the barrier keeps the scheduler from sinking these loads towards
        // their use in the next iteration (which it does to save registers)
        issue(pf[(ph + K - 1) % K], i + K - 1);
        __builtin_amdgcn_sched_barrier(0);
        // adjoint: the forward vectors of this iteration's rows, used after
        // the levels (own columns of chunk rows only)
        double2 fv[ADJ && !REV ? D : 1];
        if constexpr (ADJ && !REV) {
#pragma unroll
            for (int j = 1; j <= D; ++j) {
                const int32_t rel = i - (D - 1) - (j - 1);
                const uint32_t lanepart = rel >= 0 && rel < nrows ? s16 : kOut;
                const uint32_t ro = (uint32_t)(rr - (j - 1)) * row16 + (uint32_t)(D - j) * nb16;
                fv[j - 1] = BORDER ? bload2(rfw, ro + lanepart, 0) : bload2(rfw, lanepart, ro);
            }
        }
        lv[0][sl0] = cur.a;  // level 0, row rr+1
        if (REV) vl[0][sl0] = cur.va;
        dd[ph % RS] = op.s2 * (cur.e + op.dshift);
        if (ADJ) P[ph % RS] = cur.acc;  // gbar of row rr
#pragma unroll
        for (int j = 1; j <= D; ++j) {
            const int32_t q = rr - dir * (j - 1);
            const int32_t rel = q - ys;
            const int ps = ((ph - (j - 1)) % RS + RS) % RS;  // ring slot of row q
            // on the border a level outside its rows is zero
            const bool active =
                !BORDER || (q >= max(ys - (D - j), 0) && q <= min(ys + nrows - 1 + (D - j), W - 1));
            double2 val;
            {
                // rows q-1 (m) and q+1 (p): the oldest and newest of the window
                // walking downwards, the other way round walking upwards
                const double2 c = lv[j - 1][sl1];
                const double2 m = UP ? lv[j - 1][sl0] : lv[j - 1][sl2], p = UP ? lv[j - 1][sl2] : lv[j - 1][sl0];
                double2 s = stencil_sum(m, p, from_left0(c), from_right0(c), q);
                if (j == 1) s = cadd(s, cur.ext);
                const double d = dd[ps];
                if (HEAD && j == 1) {
                    val = make_double2(0.5 * fma(d, c.x, op.off2 * s.x), 0.5 * fma(d, c.y, op.off2 * s.y));
                } else {
                    const double2 prev = j == 1 ? cur.km1 : lv[j >= 2 ? j - 2 : 0][sl2];
                    // level D of a downward pass may be level 0 (H~ u_1 in place of 2 H~)
                    const bool half = REV && j == D;
                    const double dj = half ? d * A.hD : d, oj = half ? op.off2 * A.hD : op.off2;
                    val = make_double2(fma(dj, c.x, fma(oj, s.x, -prev.x)), fma(dj, c.y, fma(oj, s.y, -prev.y)));
                }
                if (ADJ) val = cfma(gw.g[j], P[ps], val);
                if (BORDER) val = csel(colok && active, val, zero);
                const bool mine = rel >= 0 && rel < nrows;  // a row of the chunk
                if (PROP) {
                    if (j == 1) {
                        if (HEAD) {
                            P[ps] = cfma(gw.g[1], val, cfma(gw.g[0], c, zero));
                            st2(rck, q, c, mine);
                            const bool sum = own && mine;
                            nrm += sum ? c.x * c.x + c.y * c.y : 0.0;
                            en += sum ? c.x * val.x + c.y * val.y : 0.0;
                        } else {
                            P[ps] = cfma(gw.g[1], val, cur.acc);
                        }
                    } else {
                        P[ps] = cfma(gw.g[j], val, P[ps]);
                    }
                }
                if (ALL) st2(rsrc(A.all[j - 1], nb16), q, val, mine);
                if (!ALL && j == D - 1) st2(ro1, q, val, mine);
                if (!ALL && j == D) {
                    st2(ro2, q, val, mine);
                    if (PROP) st2(racc, q, P[ps], mine);
                }
            }
            if (j < D) lv[j][sl0] = val;
            if constexpr (REV) {
                // the forward vector v_{k-j} of row q, from v_{k-j+1} and v_{k-j+2}
                const double2 c = vl[j - 1][sl1], m = vl[j - 1][sl2], p = vl[j - 1][sl0];
                double2 s = stencil_sum(m, p, from_left0(c), from_right0(c), q);
                if (j == 1) s = cadd(s, cur.vext);
                const double2 prev = j == 1 ? cur.vkm1 : vl[j >= 2 ? j - 2 : 0][sl2];
                const double d = dd[ps];
                double2 vv = make_double2(fma(d, c.x, fma(op.off2, s.x, -prev.x)),
                                          fma(d, c.y, fma(op.off2, s.y, -prev.y)));
                if (BORDER) vv = csel(colok && active, vv, zero);
                const bool mine = rel >= 0 && rel < nrows;
                if (j == D - 1) st2(rvo1, q, vv, mine);
                if (j == D) st2(rvo2, q, vv, mine);
                if (j < D) vl[j][sl0] = vv;
            }
        }
        if constexpr (ADJ) {
            // dL/dV of row rr - (j-1): level j's share, from the centre of
            // level j-1's window (u_{k-j+2}, before this iteration moved it)
            // and v_{k-j+1}; levels in order, as single-level passes add them
#pragma unroll
            for (int j = 1; j <= D; ++j) {
                const int32_t rel = i - (D - 1) - (j - 1);
                const int ps = ((ph - (j - 1)) % RS + RS) % RS;
                const double2 c = lv[j - 1][sl1];
                const double2 f = REV ? vl[REV ? j - 1 : 0][sl1] : fv[REV ? 0 : j - 1];
                const double t = c.x * f.x + c.y * f.y;
                G[ps] = (j == 1 ? cur.gr : G[ps]) + (REV && j == D ? A.gfD : A.gf) * t;
                if (j == D) st1(rgr, rr - (D - 1), G[ps], rel >= 0 && rel < nrows);
            }
        }
    };
    // Iterations: level 1 from its first needed row until level D has
    // passed the last row, in whole unrolled bodies without tests.  Those
    // past the end compute only rows below the chunk (never stored); they
    // read at most D + 1 rows past it, which the range check covers.
    const int32_t T = nrows + 2 * (D - 1);
    for (base = 0; base < T; base += U) phases<0, U>(step);
}

// The walk of one wavefront: wavefronts whose 64 lanes lie on lattice
// columns and whose every row read (ys - D up to the rows below the chunk
// that the last unrolled body loads, or walking upwards from ye - 1 + D up to
// the rows above the chunk that the last body loads) lies inside the lattice
// skip the border tests.  deep_dispatch maps the wavefronts of a grid of
// 256-thread blocks to (strip, chunk).
template <int EDGE, int D, bool HEAD, int MODE, bool NT = false>
__device__ __forceinline__ void deep_wave(const OpPair &op, int32_t strip, int32_t chunk, const DeepArgs<D> &A,
                                          double &nrm, double &en)
{
    const int32_t x0 = strip * deep_strip(D) - (D - 1);
    const int32_t ys = chunk * op.rows, ye = min(ys + op.rows, op.W);
    const int32_t it = deep_iterations(D, ye - ys);
    const bool cols = x0 >= 0 && x0 + 63 < op.L;
    if constexpr (MODE == kDeepProp && kDeepAlternate) {
        if (chunk & 1) {
            const int32_t hi = ye - 1 + D, lo = ye - 1 + (D - 1) - it - kDeepAhead;
            if (cols && lo >= 0 && hi < op.W)
                deep_walk<EDGE, D, HEAD, false, MODE, true, NT>(op, strip, chunk, A, nrm, en);
            else
                deep_walk<EDGE, D, HEAD, true, MODE, true, NT>(op, strip, chunk, A, nrm, en);
            return;
        }
    }
    const int32_t last = ys - (D - 1) + it + kDeepAhead;
    if (cols && ys - D >= 0 && last < op.W)
        deep_walk<EDGE, D, HEAD, false, MODE, false, NT>(op, strip, chunk, A, nrm, en);
    else
        deep_walk<EDGE, D, HEAD, true, MODE, false, NT>(op, strip, chunk, A, nrm, en);
}

template <int EDGE, int D, bool HEAD, int MODE, bool NT = false>
__device__ __forceinline__ void deep_dispatch(const OpPair &op, const DeepArgs<D> &A, double &nrm, double &en)
{
    const int32_t gwv =
        __builtin_amdgcn_readfirstlane(logical_block(op.xcd_remap) * 4 + (int32_t)(threadIdx.x >> 6));
    constexpr bool cf = kDeepChunkFast && MODE == kDeepProp;
    const int32_t strip = cf ? gwv / op.nchunks : gwv % op.nstrips;
    const int32_t chunk = cf ? gwv % op.nchunks : gwv / op.nstrips;
    if (chunk < op.nchunks && strip < op.nstrips)  // uniform per wavefront
        deep_wave<EDGE, D, HEAD, MODE, NT>(op, strip, chunk, A, nrm, en);
}

}  // namespace chebtd
