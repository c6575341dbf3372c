// HIP kernels of the single-system Chebyshev path (gfx950, wave64).
//
// The hot loop is the fused recursion step of Sect. 2.2 (arXiv:0907.3022):
//   v_{k+1} = 2 H~ v_k - v_{k-1}   (written over v_{k-1}),
//   acc    += gamma_{k+1} v_{k+1},
// complex128 throughout.  The stencil and CSR kernels take one row per
// thread; per row a stencil moves 88 bytes (v_k, v_{k-1}, v_{k+1}, acc read
// and write, on-site term) and the neighbour values of v_k come from the
// caches.  The matrix-free Holstein walk takes one phonon configuration per
// thread across its electron sites (eq. (ghm)).  Reductions (norm,
// energy, region sums, bounds) are deterministic: a fixed butterfly inside
// each wavefront, fixed-order sums across wavefronts and blocks, no
// floating-point atomics.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cstdint>

#include "internal.h"
#include "device_ops.h"

namespace chebtd {

// ---------------------------------------------------------------------------
// Step head: v1 = H~ v0, acc = g0 v0 + g1 v1, partial <v0|v0>, <v0|H~ v0>
// ---------------------------------------------------------------------------
__device__ __forceinline__ void head_body(int64_t i, bool valid, double2 vi, double2 h2, double2 *v1,
                                          double2 *acc, double2 g0, double2 g1, double2 *ckpt,
                                          double *partials)
{
    __shared__ double red[2 * (1024 / 64)];
    double nrm = 0.0, e = 0.0;
    if (valid) {
        const double2 h = cscale(0.5, h2);
        if (v1) {  // null: reduction only (norm and energy of v0)
            v1[i] = h;
            double2 a = make_double2(0.0, 0.0);
            a = cfma(g0, vi, a);
            a = cfma(g1, h, a);
            acc[i] = a;
        }
        if (ckpt) ckpt[i] = vi;
        nrm = vi.x * vi.x + vi.y * vi.y;
        e = vi.x * h.x + vi.y * h.y;
    }
    block_sum2(nrm, e, red);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = nrm;
        partials[2 * blockIdx.x + 1] = e;
    }
}

__global__ __launch_bounds__(kBlock) void k_head_chain(OpChain op, const double2 *__restrict__ v0,
                                                       double2 *__restrict__ v1,
                                                       double2 *__restrict__ acc, double2 g0,
                                                       double2 g1, double2 *ckpt, double *partials)
{
    const int64_t i = ChainRow::row(op);
    double2 vi = make_double2(0.0, 0.0), h2 = vi;
    if (i >= 0) {
        vi = v0[i];
        h2 = ChainRow::apply2(op, i, v0, vi);
    }
    head_body(i, i >= 0, vi, h2, v1, acc, g0, g1, ckpt, partials);
}

template <int EDGE>
__global__ __launch_bounds__(kBlock) void k_head_honey(OpHoney op, const double2 *__restrict__ v0,
                                                       double2 *__restrict__ v1,
                                                       double2 *__restrict__ acc, double2 g0,
                                                       double2 g1, double2 *ckpt, double *partials)
{
    int32_t x, y;
    const int64_t i = HoneyRow<EDGE>::row_xy(op, x, y);
    double2 vi = make_double2(0.0, 0.0), h2 = vi;
    if (i >= 0) {
        vi = v0[i];
        h2 = HoneyRow<EDGE>::apply2(op, i, x, y, v0, vi);
    }
    head_body(i, i >= 0, vi, h2, v1, acc, g0, g1, ckpt, partials);
}

__global__ __launch_bounds__(kBlock) void k_head_csr(OpCsr op, const double2 *__restrict__ v0,
                                                     double2 *__restrict__ v1,
                                                     double2 *__restrict__ acc, double2 g0,
                                                     double2 g1, double2 *ckpt, double *partials)
{
    const int64_t i = CsrRow::row(op);
    double2 vi = make_double2(0.0, 0.0), h2 = vi;
    if (i >= 0) {
        vi = v0[i];
        h2 = CsrRow::apply2(op, i, v0, vi);
    }
    head_body(i, i >= 0, vi, h2, v1, acc, g0, g1, ckpt, partials);
}

// ---------------------------------------------------------------------------
// Hot loop: v_{k+1} = 2 H~ v_k - v_{k-1} over v_{k-1}; acc += g v_{k+1}
// ---------------------------------------------------------------------------
__device__ __forceinline__ void iter_body(int64_t i, double2 h2, double2 *vprev, double2 *acc,
                                          double2 g)
{
    const double2 p = vprev[i];
    const double2 nv = csub(h2, p);
    vprev[i] = nv;
    acc[i] = cfma(g, nv, acc[i]);
}

__global__ __launch_bounds__(kBlock) void k_iter_chain(OpChain op, const double2 *__restrict__ vk,
                                                       double2 *vprev, double2 *__restrict__ acc,
                                                       double2 g)
{
    const int64_t i = ChainRow::row(op);
    if (i < 0) return;
    const double2 vi = vk[i];
    iter_body(i, ChainRow::apply2(op, i, vk, vi), vprev, acc, g);
}

template <int EDGE>
__global__ __launch_bounds__(kBlock) void k_iter_honey(OpHoney op, const double2 *__restrict__ vk,
                                                       double2 *vprev, double2 *__restrict__ acc,
                                                       double2 g)
{
    int32_t x, y;
    const int64_t i = HoneyRow<EDGE>::row_xy(op, x, y);
    if (i < 0) return;
    const double2 vi = vk[i];
    iter_body(i, HoneyRow<EDGE>::apply2(op, i, x, y, vk, vi), vprev, acc, g);
}

// Holstein recursion order, one thread per (group of electron sites,
// phonon configuration r): the thread walks its sites keeping v_k of the
// previous, current and next site in registers, so each v_k value is read
// once (the electron hops need the neighbouring sites' blocks, which lie
// nconf states apart).  Consecutive threads take consecutive r: every
// load and store of a site is contiguous across the wavefront except the
// phonon partners v(s, up_s(r)) and v(s, dn_s(r)).
// Thread t = grp * nconf + r covers sites [grp*spt, min(grp*spt + spt, L)).
//
// The accumulator is brought up to date only every third order (and at the
// step's last): the pass forming v_{k+1} holds v_{k-1} (read before v_{k+1}
// overwrites it), v_k and v_{k+1}, so it can add the weights of up to those
// three orders at once; the other passes neither read nor write acc (57 of
// the 89 B per state).  nacc = 0..3 terms: acc += ga v_{k-1} + gb v_k +
// gc v_{k+1} with the leading terms dropped.
//
// RANK: the thread ranks the partners itself instead of reading the
// per-state tables (9 B per state fewer).  Configurations of total T are
// ranked by the combinatorial number system,
//   rank(n) = C(T-1+L, L) + sum_{j<L-1} t_j,
//   t_j = C(l_j + m_j, m_j) - C(l_j - n_j + m_j, m_j),
// with l_j = T - n_0 - .. - n_{j-1} phonons left and m_j = L-1-j parts after
// j.  n + e_s changes l_j by +1 for j <= s and leaves the terms past s
// alone, so rank(n + e_s) = r + C(T+L-1, L-1) + sum_{j<s} (u_j - t_j)
// + x_s - t_s, with u_j, x_s the terms at l_j + 1 (and n_s + 1 at s); and
// rank(n - e_s) = r - C(T+L-2, L-1) + sum_{j<s} (d_j - t_j) + y_s - t_s at
// l_j - 1.  Walking the sites in order, the thread takes the digits n_s
// from r as it goes (unranking) and carries the two prefix sums.
//
// hol_walk is one thread's walk: configuration r, sites [s0, s1).
template <bool RANK, bool HEAD>
__device__ __forceinline__ void hol_walk(const OpHol &op, int spt, int brows, const int32_t *sbin, uint32_t lb,
                                         uint32_t C, const double2 *__restrict__ vk, double2 *vprev,
                                         double2 *__restrict__ acc, int nacc, double2 ga, double2 gb, double2 gc,
                                         double2 *ckpt, double &nrm, double &en)
{
    const int32_t L = op.L, K = L + 1;  // binomial table: brows x (L + 1)
    // C(a, m) from the table; zero outside it
    auto cb = [&](int32_t a, int32_t m) -> int32_t {
        return (a < 0 || a >= brows || m < 0 || m > L) ? 0 : sbin[a * K + m];
    };
    const uint32_t Lu = (uint32_t)L;
    // (grp, r) from t: one division per wavefront, then at most a few steps
    const uint32_t b0 = lb * blockDim.x;
    const uint64_t t = (uint64_t)b0 + threadIdx.x;
    uint32_t grp = __builtin_amdgcn_readfirstlane(b0 / C);
    uint32_t r = (uint32_t)t - grp * C;
    while (r >= C) {
        r -= C;
        ++grp;
    }
    const uint32_t s0 = grp * (uint32_t)spt, s1 = min(s0 + (uint32_t)spt, Lu);
    const double2 zero = make_double2(0.0, 0.0);
    // RANK state: total T, phonons left, rank within the shell still to
    // account for, and the two prefix sums of the partner ranks
    int32_t T = 0, left = 0;
    uint32_t within = 0;
    int64_t dup = 0, ddn = 0;
    // digit s of the configuration (unranking) and its term t_s; the prefix
    // sums then take site s
    auto digit = [&](int32_t s, int32_t &ns, int32_t &ts) {
        if (s + 1 < L) {
            const int32_t m = L - 1 - s;
            const int32_t all = cb(left + m, m);
            int32_t v = 0;
            while (v < left && (uint32_t)(all - cb(left - (v + 1) + m, m)) <= within) ++v;
            ts = all - cb(left - v + m, m);
            within -= (uint32_t)ts;
            ns = v;
        } else {
            ns = left;
            ts = 0;
        }
    };
    auto advance = [&](int32_t s, int32_t ns, int32_t ts) {
        if (s + 1 < L) {
            const int32_t m = L - 1 - s;
            dup += (int64_t)(cb(left + 1 + m, m) - cb(left + 1 - ns + m, m)) - ts;
            ddn += (int64_t)(cb(left - 1 + m, m) - cb(left - 1 - ns + m, m)) - ts;
        }
        left -= ns;
    };
    double wt;
    if constexpr (RANK) {
        while (T < (int32_t)brows - L - 2 && (uint32_t)cb(T + L, L) <= r) ++T;  // brows - L - 2 = nph
        within = r - (T == 0 ? 0u : (uint32_t)cb(T - 1 + L, L));
        left = T;
        for (int32_t s = 0; s < (int32_t)s0; ++s) {  // digits before the group
            int32_t ns, ts;
            digit(s, ns, ts);
            advance(s, ns, ts);
        }
        wt = op.w0 * (double)T - op.b;
    } else {
        wt = op.w0 * (double)op.tot[r] - op.b;
    }
    const bool can_up = RANK && T < (int32_t)brows - L - 2;
    const int64_t up0 = RANK ? (int64_t)r + cb(T + L - 1, L - 1) : 0;
    const int64_t dn0 = RANK ? (int64_t)r - cb(T + L - 2, L - 1) : 0;
    // v_k at sites s-1, s, s+1 of configuration r
    double2 left_v = zero;
    if (s0 > 0)
        left_v = vk[(size_t)(s0 - 1) * C + r];
    else if (op.periodic)
        left_v = vk[(size_t)(Lu - 1) * C + r];
    double2 cur = vk[(size_t)s0 * C + r];
    for (uint32_t s = s0; s < s1; ++s) {
        const size_t i = (size_t)s * C + r;
        double2 right = zero;
        if (s + 1 < Lu)
            right = vk[i + C];
        else if (op.periodic)
            right = vk[r];
        int32_t ru, rd;
        uint32_t ni;
        if constexpr (RANK) {
            int32_t ns, ts;
            const int32_t si = (int32_t)s;
            digit(si, ns, ts);
            int64_t xs = 0, ys = 0;
            if (si + 1 < L) {
                const int32_t m = L - 1 - si;
                xs = (int64_t)(cb(left + 1 + m, m) - cb(left - ns + m, m)) - ts;
                ys = (int64_t)(cb(left - 1 + m, m) - cb(left - ns + m, m)) - ts;
            }
            ru = can_up ? (int32_t)(up0 + dup + xs) : -1;
            rd = ns > 0 ? (int32_t)(dn0 + ddn + ys) : -1;
            ni = (uint32_t)ns;
            advance(si, ns, ts);
        } else {
            ru = op.up[i];
            rd = op.dn[i];
            ni = op.occ[i];
        }
        const size_t base = (size_t)s * C;
        double px = 0.0, py = 0.0;
        if (ru >= 0) {
            const double2 u = vk[base + (uint32_t)ru];
            const double w = op.sq[ni + 1];
            px = fma(w, u.x, px);
            py = fma(w, u.y, py);
        }
        if (rd >= 0) {
            const double2 u = vk[base + (uint32_t)rd];
            const double w = op.sq[ni];
            px = fma(w, u.x, px);
            py = fma(w, u.y, py);
        }
        const double d = op.Delta[s] + wt, gw = op.gw0[s];
        // hops: left and right are zero where an open chain ends
        const double hx = left_v.x + right.x, hy = left_v.y + right.y;
        const double hvx = fma(d, cur.x, fma(-op.t, hx, -gw * px));
        const double hvy = fma(d, cur.y, fma(-op.t, hy, -gw * py));
        if constexpr (HEAD) {
            const double2 h = make_double2(0.5 * (op.s2 * hvx), 0.5 * (op.s2 * hvy));
            if (vprev) {  // null: reduction only (norm and energy of v0)
                vprev[i] = h;
                acc[i] = cfma(gb, h, cfma(ga, cur, zero));
            }
            if (ckpt) ckpt[i] = cur;
            nrm += cur.x * cur.x + cur.y * cur.y;
            en += cur.x * h.x + cur.y * h.y;
        } else {
            const double2 p = vprev[i];
            const double2 nv = csub(make_double2(op.s2 * hvx, op.s2 * hvy), p);
            vprev[i] = nv;
            if (nacc > 0) {  // uniform across the launch
                double2 a = acc[i];
                if (nacc >= 3) a = cfma(ga, p, a);
                if (nacc >= 2) a = cfma(gb, cur, a);
                acc[i] = cfma(gc, nv, a);
            }
        }
        left_v = cur;
        cur = right;
    }
}

// HEAD: the same walk as the step head, v1 = H~ v0 (into vprev, which is not
// read; null: reduction only), acc = ga v0 + gb v1, ckpt = v0 (if given),
// and per block the partial sums <v0|v0>, <v0|H~ v0> into partials (one
// pair per block: the sum over a block's configurations and their sites).
template <bool RANK, bool HEAD>
__global__ __launch_bounds__(kBlock) void k_iter_hol(OpHol op, int spt, int remap, const int32_t *binom,
                                                     int brows, const double2 *__restrict__ vk, double2 *vprev,
                                                     double2 *__restrict__ acc, int nacc, double2 ga, double2 gb,
                                                     double2 gc, double2 *ckpt, double *partials)
{
    extern __shared__ int32_t sbin[];
    __shared__ double red[2 * (kBlock / 64)];
    const int32_t L = op.L, K = L + 1;  // binomial table: brows x (L + 1)
    if constexpr (RANK) {
        for (int q = threadIdx.x; q < brows * K; q += blockDim.x) sbin[q] = binom[q];
        __syncthreads();
    }
    const uint32_t C = op.nconf, Lu = (uint32_t)L;
    const uint32_t ngrp = (Lu + (uint32_t)spt - 1) / (uint32_t)spt;
    // remap: each XCD takes one contiguous range of configurations, so the
    // phonon partners that neighbouring wavefronts share meet in one L2
    const uint32_t lb = (uint32_t)logical_block(remap);
    const uint64_t t = (uint64_t)lb * blockDim.x + threadIdx.x;
    double nrm = 0.0, en = 0.0;  // HEAD: this thread's share of <v0|v0>, <v0|H~ v0>
    if (t < (uint64_t)C * ngrp) {
        hol_walk<RANK, HEAD>(op, spt, brows, sbin, lb, C, vk, vprev, acc, nacc, ga, gb, gc, ckpt, nrm, en);
    }
    if constexpr (HEAD) {
        block_sum2(nrm, en, red);
        if (threadIdx.x == 0) {
            partials[2 * blockIdx.x] = nrm;
            partials[2 * blockIdx.x + 1] = en;
        }
    }
}

// The accumulator as in the Holstein walk: up to three orders' weights at
// once (nacc terms), none on the other orders.
__global__ __launch_bounds__(kBlock) void k_iter_csr(OpCsr op, const double2 *__restrict__ vk,
                                                     double2 *vprev, double2 *__restrict__ acc, int nacc,
                                                     double2 ga, double2 gb, double2 gc)
{
    const int64_t i = CsrRow::row(op);
    if (i < 0) return;
    const double2 vi = vk[i];
    const double2 h2 = CsrRow::apply2(op, i, vk, vi);
    const double2 p = vprev[i];
    const double2 nv = csub(h2, p);
    vprev[i] = nv;
    if (nacc > 0) {  // uniform across the launch
        double2 a = acc[i];
        if (nacc >= 3) a = cfma(ga, p, a);
        if (nacc >= 2) a = cfma(gb, vi, a);
        acc[i] = cfma(gc, nv, a);
    }
}

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
// One block: fixed-order sums of (norm, <v0|H~v0>) partials; writes the
// values for step counter[0] and advances the counter.
__global__ __launch_bounds__(256) void k_finalize_ne(const double *__restrict__ partials, int nparts,
                                                     double a, double b, double *norm_out,
                                                     double *energy_out, int64_t *counter,
                                                     double *dst2)
{
    __shared__ double red[2 * 4];
    NeFinal f{partials, nparts, a, b, norm_out, energy_out, counter};
    finalize_ne_block(f, dst2, red);
}

__global__ void k_reset_counter(int64_t *counter) { counter[0] = 0; }

// Norm and region sums: each thread sums the sites i = t, t + stride, ... in
// order (stride = the grid's thread count, at most kReduceBlocks blocks), so
// the final one-block sum reads few partials whatever n is; fixed order.
__global__ __launch_bounds__(kBlock) void k_norm(const double2 *__restrict__ psi, int64_t n,
                                                 double *partials)
{
    __shared__ double red[2 * (kBlock / 64)];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double s = 0.0, z = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double2 v = psi[i];
        s += v.x * v.x + v.y * v.y;
    }
    block_sum2(s, z, red);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s;
        partials[2 * blockIdx.x + 1] = 0.0;
    }
}

__global__ __launch_bounds__(kBlock) void k_region(const double2 *__restrict__ psi,
                                                   const uint8_t *__restrict__ mask, int64_t n,
                                                   double *partials)
{
    __shared__ double red[2 * (kBlock / 64)];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double s = 0.0, z = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (mask[i]) {
            const double2 v = psi[i];
            s += v.x * v.x + v.y * v.y;
        }
    }
    block_sum2(s, z, red);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s;
        partials[2 * blockIdx.x + 1] = 0.0;
    }
}

// out[0] = sum of partials[2p], out[1] = sum of partials[2p+1] (fixed order)
__global__ __launch_bounds__(256) void k_sum_partials(const double *__restrict__ partials,
                                                      int nparts, double *out)
{
    __shared__ double red[2 * 4];
    double s0 = 0.0, s1 = 0.0;
    for (int p = threadIdx.x; p < nparts; p += blockDim.x) {
        s0 += partials[2 * p];
        s1 += partials[2 * p + 1];
    }
    block_sum2(s0, s1, red);
    if (threadIdx.x == 0) {
        out[0] = s0;
        out[1] = s1;
    }
}

__global__ __launch_bounds__(kBlock) void k_density(const double2 *__restrict__ psi,
                                                    double *__restrict__ rho, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const double2 v = psi[i];
        rho[i] = v.x * v.x + v.y * v.y;
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_zero(double *p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0;
}

// dst = g src (src may equal dst)
__global__ __launch_bounds__(kBlock) void k_scale_copy(const double2 *src, double2 *dst, double2 g,
                                                       int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        double2 a = make_double2(0.0, 0.0);
        dst[i] = cfma(g, src[i], a);
    }
}

// ---------------------------------------------------------------------------
// CSR structure check (run once when a caller hands in a matrix): flag[0] is
// set if rowptr is not a non-decreasing map from [0, n] onto [0, nnz] or a
// column index falls outside [0, n).  Columns are read only inside a row
// whose bounds were verified first.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_csr_check(const int64_t *__restrict__ rowptr,
                                                      const int32_t *__restrict__ col, int64_t n,
                                                      int64_t nnz, int64_t *flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t p0 = rowptr[i], p1 = rowptr[i + 1];
    bool bad = p0 < 0 || p1 < p0 || p1 > nnz;
    if (i == 0 && p0 != 0) bad = true;
    if (i == n - 1 && p1 != nnz) bad = true;
    if (!bad) {
        for (int64_t p = p0; p < p1; ++p) {
            const int32_t c = col[p];
            if (c < 0 || (int64_t)c >= n) bad = true;
        }
    }
    if (bad) flag[0] = 1;
}

__global__ void k_clear_flag(int64_t *flag) { flag[0] = 0; }

hipError_t launch_csr_check(hipStream_t s, const int64_t *rowptr, const int32_t *col, int64_t n,
                            int64_t nnz, int64_t *flag)
{
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, s, flag);
    const int64_t nb = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_csr_check, dim3((unsigned)nb), dim3(kBlock), 0, s, rowptr, col, n, nnz, flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gershgorin discs: per block (min(H_ii - R_i), max(H_ii + R_i))
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_minmax(double &lo, double &hi, double *lds)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, o, 64));
        hi = fmax(hi, __shfl_xor(hi, o, 64));
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) {
        lds[2 * w] = lo;
        lds[2 * w + 1] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) {
            lo = fmin(lo, lds[2 * i]);
            hi = fmax(hi, lds[2 * i + 1]);
        }
    }
}

struct GershSrc {
    int kind;  // 0 chain, 1 honeycomb zigzag, 2 honeycomb armchair, 3 csr, 4 Holstein tables
    OpHol hol;
    int64_t n;
    const double *onsite;  // V or eps
    double dx;
    double t;
    int32_t W, L;
    const int64_t *rowptr;
    const int32_t *col;
    const double2 *val;
};

__global__ __launch_bounds__(kBlock) void k_gersh(GershSrc g, double *partials)
{
    __shared__ double red[2 * (kBlock / 64)];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double lo = INFINITY, hi = -INFINITY;
    if (i < g.n) {
        double d = 0.0, r = 0.0;
        if (g.kind == 0) {
            const double inv = 1.0 / (g.dx * g.dx), h = 0.5 / (g.dx * g.dx);
            d = inv + g.onsite[i];
            if (i > 0) r += h;
            if (i + 1 < g.n) r += h;
        } else if (g.kind == 1 || g.kind == 2) {
            const int32_t y = (int32_t)(i / g.L), x = (int32_t)(i - (int64_t)y * g.L);
            const bool even = ((x + y) & 1) == 0;
            int nb = 0;
            if (g.kind == 1) {
                nb += (x > 0) + (x + 1 < g.L);
                nb += even ? (y + 1 < g.W) : (y > 0);
            } else {
                nb += (y > 0) + (y + 1 < g.W);
                nb += even ? (x + 1 < g.L) : (x > 0);
            }
            d = g.onsite[i];
            for (int q = 0; q < nb; ++q) r += fabs(g.t);
        } else if (g.kind == 4) {
            const OpHol &h = g.hol;
            const uint32_t L = (uint32_t)h.L;
            uint32_t site, cfg;
            HolRow::split(h, i, site, cfg);
            d = h.Delta[site] + h.w0 * (double)h.tot[cfg];
            const int hops = h.periodic ? 2 : (site > 0) + (site + 1 < L);
            r = hops * fabs(h.t);
            const uint32_t ni = h.occ[i];
            const double gw = fabs(h.gw0[site]);
            if (h.up[i] >= 0) r += gw * h.sq[ni + 1];
            if (h.dn[i] >= 0) r += gw * h.sq[ni];
        } else {
            for (int64_t p = g.rowptr[i]; p < g.rowptr[i + 1]; ++p) {
                const double2 h = g.val[p];
                if (g.col[p] == i)
                    d += h.x;
                else
                    r += sqrt(h.x * h.x + h.y * h.y);
            }
        }
        lo = d - r;
        hi = d + r;
    }
    block_minmax(lo, hi, red);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = lo;
        partials[2 * blockIdx.x + 1] = hi;
    }
}

__global__ __launch_bounds__(256) void k_minmax_final(const double *partials, int nparts,
                                                      double *out2)
{
    __shared__ double red[2 * 4];
    double lo = INFINITY, hi = -INFINITY;
    for (int p = threadIdx.x; p < nparts; p += blockDim.x) {
        lo = fmin(lo, partials[2 * p]);
        hi = fmax(hi, partials[2 * p + 1]);
    }
    block_minmax(lo, hi, red);
    if (threadIdx.x == 0) {
        out2[0] = lo;
        out2[1] = hi;
    }
}

// ---------------------------------------------------------------------------
// Holstein observables (Fig. 3): one thread per phonon configuration r; the
// L states (s, r) sit nconf apart, so a wavefront reads contiguous runs.
// Per site s the block reduces
//   <n_s>        += |psi(s,r)|^2
//   <b_s^+ b_s>  += n_s(r) * sum_j |psi(j,r)|^2
//   chi_ss       += 2 Re[conj(psi(s,r)) sqrt(n_s(r)+1) psi(s, up_s(r))]
// into partials[block][3L].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_holstein_obs(const double2 *__restrict__ psi,
                                                         const uint8_t *__restrict__ occ,
                                                         const int32_t *__restrict__ up,
                                                         int64_t nconf, int L, double *partials)
{
    __shared__ double red[2 * (kBlock / 64)];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = r < nconf;
    double w = 0.0;
    if (valid) {
        for (int j = 0; j < L; ++j) {
            const double2 v = psi[(int64_t)j * nconf + r];
            w += v.x * v.x + v.y * v.y;
        }
    }
    for (int s = 0; s < L; ++s) {
        double dn = 0.0, dph = 0.0, dchi = 0.0;
        if (valid) {
            const int64_t i = (int64_t)s * nconf + r;
            const double2 v = psi[i];
            const int ns = occ[i];
            dn = v.x * v.x + v.y * v.y;
            dph = ns * w;
            const int32_t ru = up[i];
            if (ru >= 0) {
                const double2 u = psi[(int64_t)s * nconf + ru];
                dchi = 2.0 * sqrt((double)ns + 1.0) * (v.x * u.x + v.y * u.y);
            }
        }
        block_sum2(dn, dph, red);
        __syncthreads();
        double z = 0.0;
        block_sum2(dchi, z, red);
        __syncthreads();
        if (threadIdx.x == 0) {
            double *dst = partials + (size_t)blockIdx.x * 3 * L;
            dst[s] = dn;
            dst[L + s] = dph;
            dst[2 * L + s] = dchi;
        }
    }
}

// One block per output o of the 3L: fixed-order sum of partials[p][o].
__global__ __launch_bounds__(256) void k_holstein_obs_final(const double *partials, int nparts, int L,
                                                            double *n_out, double *nph_out, double *chi_out)
{
    __shared__ double red[2 * 4];
    const int o = blockIdx.x;
    double s = 0.0, z = 0.0;
    for (int p = threadIdx.x; p < nparts; p += blockDim.x) s += partials[(size_t)p * 3 * L + o];
    block_sum2(s, z, red);
    if (threadIdx.x == 0) {
        if (o < L)
            n_out[o] = s;
        else if (o < 2 * L)
            nph_out[o - L] = s;
        else
            chi_out[o - 2 * L] = s;
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
int64_t grid_blocks(const Ctx &c)
{
    if (c.kind == HKind::Honeycomb) return c.W * ((c.L + kBlock - 1) / kBlock);
    return (c.n + kBlock - 1) / kBlock;
}

// Electron sites per thread of the Holstein walk (measured on MI355X with the
// XCD-contiguous order and acc every third order): all of them (L = 10 ring:
// 23.2 us per order against 24.4 for groups of five; L = 18 polaron: 10.60 ms
// against 10.82 for groups of nine and 10.88 for six); hol_spt > 0 groups them
static int hol_sites_per_thread(const Ctx &c)
{
    return c.hol_spt > 0 ? (int)std::min<int64_t>(c.hol_spt, c.hol_L) : (int)c.hol_L;
}

static int64_t hol_walk_blocks(const Ctx &c)
{
    const int64_t L = c.hol_L, spt = hol_sites_per_thread(c);
    return (c.hol_nconf * ((L + spt - 1) / spt) + kBlock - 1) / kBlock;
}

// The Holstein walk, as an order of the recursion or (head) as the step head.
static hipError_t launch_hol_walk(const Ctx &c, hipStream_t s, bool head, const double2 *vk, double2 *vprev,
                                  double2 *acc, int nacc, double2 ga, double2 gb, double2 gc, double2 *ckpt,
                                  double *partials)
{
    const int spt = hol_sites_per_thread(c);
    const dim3 grid((unsigned)hol_walk_blocks(c)), block(kBlock);
    if (c.hol_brows > 0) {
        const size_t lds = (size_t)c.hol_brows * (size_t)(c.hol_L + 1) * sizeof(int32_t);
        const int32_t *bin = static_cast<const int32_t *>(c.hol_binom.p);
        if (head)
            hipLaunchKernelGGL((k_iter_hol<true, true>), grid, block, lds, s, make_hol(c), spt, c.hol_remap, bin,
                               c.hol_brows, vk, vprev, acc, 0, ga, gb, gc, ckpt, partials);
        else
            hipLaunchKernelGGL((k_iter_hol<true, false>), grid, block, lds, s, make_hol(c), spt, c.hol_remap, bin,
                               c.hol_brows, vk, vprev, acc, nacc, ga, gb, gc, nullptr, nullptr);
    } else {
        if (head)
            hipLaunchKernelGGL((k_iter_hol<false, true>), grid, block, 0, s, make_hol(c), spt, c.hol_remap, nullptr,
                               0, vk, vprev, acc, 0, ga, gb, gc, ckpt, partials);
        else
            hipLaunchKernelGGL((k_iter_hol<false, false>), grid, block, 0, s, make_hol(c), spt, c.hol_remap,
                               nullptr, 0, vk, vprev, acc, nacc, ga, gb, gc, nullptr, nullptr);
    }
    return hipGetLastError();
}

int64_t head_blocks(const Ctx &c)
{
    return c.kind == HKind::Holstein ? hol_walk_blocks(c) : grid_blocks(c);
}

hipError_t launch_head(const Ctx &c, hipStream_t s, const double2 *v0, double2 *v1, double2 *acc,
                       double2 g0, double2 g1, double2 *ckpt, double *partials)
{
    if (c.kind == HKind::Holstein)
        return launch_hol_walk(c, s, true, v0, v1, acc, 0, g0, g1, make_double2(0.0, 0.0), ckpt, partials);
    const dim3 grid((unsigned)grid_blocks(c)), block(kBlock);
    switch (c.kind) {
    case HKind::Chain:
        hipLaunchKernelGGL(k_head_chain, grid, block, 0, s, make_chain(c), v0, v1, acc, g0, g1, ckpt,
                           partials);
        break;
    case HKind::Honeycomb:
        if (c.edge == CHEBTD_ZIGZAG)
            hipLaunchKernelGGL(k_head_honey<CHEBTD_ZIGZAG>, grid, block, 0, s, make_honey(c), v0, v1,
                               acc, g0, g1, ckpt, partials);
        else
            hipLaunchKernelGGL(k_head_honey<CHEBTD_ARMCHAIR>, grid, block, 0, s, make_honey(c), v0,
                               v1, acc, g0, g1, ckpt, partials);
        break;
    case HKind::Csr:
        hipLaunchKernelGGL(k_head_csr, grid, block, 0, s, make_csr(c), v0, v1, acc, g0, g1, ckpt,
                           partials);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_iter(const Ctx &c, hipStream_t s, const double2 *vk, double2 *vprev,
                       double2 *acc, double2 g)
{
    const dim3 grid((unsigned)grid_blocks(c)), block(kBlock);
    switch (c.kind) {
    case HKind::Chain:
        hipLaunchKernelGGL(k_iter_chain, grid, block, 0, s, make_chain(c), vk, vprev, acc, g);
        break;
    case HKind::Honeycomb:
        if (c.edge == CHEBTD_ZIGZAG)
            hipLaunchKernelGGL(k_iter_honey<CHEBTD_ZIGZAG>, grid, block, 0, s, make_honey(c), vk,
                               vprev, acc, g);
        else
            hipLaunchKernelGGL(k_iter_honey<CHEBTD_ARMCHAIR>, grid, block, 0, s, make_honey(c), vk,
                               vprev, acc, g);
        break;
    case HKind::Csr:
    case HKind::Holstein:
        return launch_iter_lazy(c, s, vk, vprev, acc, 1, make_double2(0.0, 0.0), make_double2(0.0, 0.0), g);
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_iter_lazy(const Ctx &c, hipStream_t s, const double2 *vk, double2 *vprev, double2 *acc, int nacc,
                            double2 ga, double2 gb, double2 gc)
{
    if ((c.kind != HKind::Holstein && c.kind != HKind::Csr) || nacc < 0 || nacc > 3) return hipErrorInvalidValue;
    if (c.kind == HKind::Csr) {
        hipLaunchKernelGGL(k_iter_csr, dim3((unsigned)grid_blocks(c)), dim3(kBlock), 0, s, make_csr(c), vk, vprev, acc,
                           nacc, ga, gb, gc);
        return hipGetLastError();
    }
    return launch_hol_walk(c, s, false, vk, vprev, acc, nacc, ga, gb, gc, nullptr, nullptr);
}

hipError_t launch_finalize_ne(hipStream_t s, const double *partials, int nparts, double a, double b,
                              double *norm_out, double *energy_out, int64_t *step_counter,
                              double *dst2)
{
    hipLaunchKernelGGL(k_finalize_ne, dim3(1), dim3(256), 0, s, partials, nparts, a, b, norm_out,
                       energy_out, step_counter, dst2);
    return hipGetLastError();
}

hipError_t launch_reset_counter(hipStream_t s, int64_t *counter)
{
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, counter);
    return hipGetLastError();
}

hipError_t launch_norm(const Ctx &c, hipStream_t s, const double2 *psi, double *partials)
{
    const int64_t nb = reduce_blocks(c.n);
    hipLaunchKernelGGL(k_norm, dim3((unsigned)nb), dim3(kBlock), 0, s, psi, c.n, partials);
    return hipGetLastError();
}

hipError_t launch_sum_partials(hipStream_t s, const double *partials, int nparts, int stride,
                               double *out)
{
    (void)stride;
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partials, nparts, out);
    return hipGetLastError();
}

hipError_t launch_copy(hipStream_t s, const double2 *src, double2 *dst, int64_t n)
{
    return hipMemcpyAsync(dst, src, (size_t)n * sizeof(double2), hipMemcpyDeviceToDevice, s);
}

hipError_t launch_scale_copy(hipStream_t s, const double2 *src, double2 *dst, double2 g, int64_t n)
{
    const int64_t nb = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_scale_copy, dim3((unsigned)nb), dim3(kBlock), 0, s, src, dst, g, n);
    return hipGetLastError();
}

hipError_t launch_density(hipStream_t s, const double2 *psi, double *rho, int64_t n)
{
    const int64_t nb = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_density, dim3((unsigned)nb), dim3(kBlock), 0, s, psi, rho, n);
    return hipGetLastError();
}

hipError_t launch_region(hipStream_t s, const double2 *psi, const uint8_t *mask, int64_t n,
                         double *partials, double *out)
{
    const int64_t nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_region, dim3((unsigned)nb), dim3(kBlock), 0, s, psi, mask, n, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partials, (int)nb, out);
    return hipGetLastError();
}

hipError_t launch_gershgorin(const Ctx &c, hipStream_t s, double *partials, double *out2)
{
    GershSrc g{};
    g.n = c.n;
    switch (c.kind) {
    case HKind::Chain:
        g.kind = 0;
        g.onsite = c.V;
        g.dx = c.dx;
        break;
    case HKind::Honeycomb:
        g.kind = c.edge == CHEBTD_ZIGZAG ? 1 : 2;
        g.onsite = c.eps;
        g.t = c.t_hop;
        g.W = (int32_t)c.W;
        g.L = (int32_t)c.L;
        break;
    case HKind::Csr:
        g.kind = 3;
        g.rowptr = c.rowptr;
        g.col = c.col;
        g.val = reinterpret_cast<const double2 *>(c.val);
        break;
    case HKind::Holstein:
        g.kind = 4;
        g.hol = make_hol(c);
        break;
    default:
        return hipErrorInvalidValue;
    }
    const int64_t nb = (c.n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_gersh, dim3((unsigned)nb), dim3(kBlock), 0, s, g, partials);
    hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(256), 0, s, partials, (int)nb, out2);
    return hipGetLastError();
}

int holstein_obs_blocks(int64_t nconf) { return (int)((nconf + kBlock - 1) / kBlock); }

hipError_t launch_holstein_obs(hipStream_t s, const double2 *psi, const uint8_t *occ,
                               const int32_t *up, int64_t nconf, int L, double *partials,
                               double *n_out, double *nph_out, double *chi_out)
{
    const int nb = holstein_obs_blocks(nconf);
    hipLaunchKernelGGL(k_holstein_obs, dim3((unsigned)nb), dim3(kBlock), 0, s, psi, occ, up, nconf, L,
                       partials);
    hipLaunchKernelGGL(k_holstein_obs_final, dim3(3 * L), dim3(256), 0, s, partials, nb, L, n_out, nph_out,
                       chi_out);
    return hipGetLastError();
}

hipError_t launch_fill_zero(hipStream_t s, double *p, int64_t count)
{
    const int64_t nb = (count + kBlock - 1) / kBlock;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)nb), dim3(kBlock), 0, s, p, count);
    return hipGetLastError();
}

}  // namespace chebtd
