// Device-side building blocks shared by the HIP kernels: complex helpers,
// deterministic wavefront/block sums, and the row mapping plus 2 H~
// application of each Hamiltonian form (chain, honeycomb brick wall, CSR).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace chebtd {

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
// Global-memory access through pointers the compiler cannot prove global
// (read from a descriptor in memory, or passed through several layers):
// addressing the data through address-space-1 pointers gives global loads
// and stores instead of flat ones.
typedef __attribute__((address_space(1))) const double *gconst_f64;
typedef __attribute__((address_space(1))) double *g_f64;
__device__ __forceinline__ double2 ldg(const double2 *p, int64_t i)
{
    const gconst_f64 q = (gconst_f64)p;
    return make_double2(q[2 * i], q[2 * i + 1]);
}
__device__ __forceinline__ double ldg(const double *p, int64_t i) { return ((gconst_f64)p)[i]; }
__device__ __forceinline__ void stg(double *p, int64_t i, double v) { ((g_f64)p)[i] = v; }
__device__ __forceinline__ void stg(double2 *p, int64_t i, double2 v)
{
    const g_f64 q = (g_f64)p;
    q[2 * i] = v.x;
    q[2 * i + 1] = v.y;
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
// a += g * v
__device__ __forceinline__ double2 cfma(double2 g, double2 v, double2 a)
{
    a.x = fma(g.x, v.x, fma(-g.y, v.y, a.x));
    a.y = fma(g.x, v.y, fma(g.y, v.x, a.y));
    return a;
}

__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Sum (a, b) over the block; thread 0 receives the totals.  lds: 2 * nwaves.
__device__ __forceinline__ void block_sum2(double &a, double &b, double *lds)
{
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) {
        lds[2 * w] = a;
        lds[2 * w + 1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) {
            sa += lds[2 * i];
            sb += lds[2 * i + 1];
        }
        a = sa;
        b = sb;
    }
}

// ---------------------------------------------------------------------------
// Row mapping and 2 H~ application per operator
// ---------------------------------------------------------------------------
struct ChainRow {
    __device__ static __forceinline__ int64_t row(const OpChain &op)
    {
        const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        return i < op.n ? i : -1;
    }
    __device__ static __forceinline__ double2 apply2(const OpChain &op, int64_t i, const double2 *v,
                                                     double2 vi)
    {
        const double d = op.s2 * (op.V[i] + op.dsh);
        double2 s = make_double2(0.0, 0.0);
        if (i > 0) s = v[i - 1];
        if (i + 1 < op.n) s = cadd(s, v[i + 1]);
        return make_double2(fma(d, vi.x, op.off2 * s.x), fma(d, vi.y, op.off2 * s.y));
    }
};

// Logical block index; with xcd_remap the blocks that one XCD receives under
// round-robin dispatch cover one contiguous range of the grid, so vertical
// neighbours of a tile are mostly cached in the same L2.
__device__ __forceinline__ int32_t logical_block(int32_t remap)
{
    const int32_t b = blockIdx.x, nb = gridDim.x;
    if (!remap) return b;
    const int32_t xcd = b & 7, slot = b >> 3;
    const int32_t per = nb >> 3, rem = nb & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + slot;
}

// The per-step norm and energy from the step head's block partials, summed
// in a fixed order by one 256-thread block (the same bits whichever kernel
// runs it): norm_out/energy_out[counter[0]] and counter[0]++, or dst2[0..1].
struct NeFinal {
    const double *partials;
    int nparts;
    double a, b;
    double *norm_out, *energy_out;
    int64_t *counter;
};

__device__ __forceinline__ void finalize_ne_block(const NeFinal &f, double *dst2, double *red)
{
    double s0 = 0.0, s1 = 0.0;
    for (int p = threadIdx.x; p < f.nparts; p += blockDim.x) {
        s0 += f.partials[2 * p];
        s1 += f.partials[2 * p + 1];
    }
    block_sum2(s0, s1, red);
    if (threadIdx.x == 0) {
        const double energy = f.a * s1 + f.b * s0;
        if (f.counter) {
            const int64_t st = f.counter[0];
            if (f.norm_out) f.norm_out[st] = s0;
            if (f.energy_out) f.energy_out[st] = energy;
            f.counter[0] = st + 1;
        }
        if (dst2) {
            dst2[0] = s0;
            dst2[1] = energy;
        }
    }
}

template <int EDGE>
struct HoneyRow {
    __device__ static __forceinline__ int64_t row_xy(const OpHoney &op, int32_t &x, int32_t &y)
    {
        const int32_t lb = logical_block(op.xcd_remap);
        y = lb / op.xblocks;
        x = (lb - y * op.xblocks) * (int32_t)blockDim.x + (int32_t)threadIdx.x;
        if (x >= op.L) return -1;
        return (int64_t)y * op.L + x;
    }
    __device__ static __forceinline__ double2 apply2(const OpHoney &op, int64_t i, int32_t x,
                                                     int32_t y, const double2 *v, double2 vi)
    {
        const double d = op.s2 * (ldg(op.eps, i) - op.b);
        double2 s = make_double2(0.0, 0.0);
        const bool even = ((x + y) & 1) == 0;
        if (EDGE == CHEBTD_ZIGZAG) {
            if (x > 0) s = ldg(v, i - 1);
            if (x + 1 < op.L) s = cadd(s, ldg(v, i + 1));
            if (even) {
                if (y + 1 < op.W) s = cadd(s, ldg(v, i + op.L));
            } else {
                if (y > 0) s = cadd(s, ldg(v, i - op.L));
            }
        } else {
            if (y > 0) s = ldg(v, i - op.L);
            if (y + 1 < op.W) s = cadd(s, ldg(v, i + op.L));
            if (even) {
                if (x + 1 < op.L) s = cadd(s, ldg(v, i + 1));
            } else {
                if (x > 0) s = cadd(s, ldg(v, i - 1));
            }
        }
        return make_double2(fma(d, vi.x, op.off2 * s.x), fma(d, vi.y, op.off2 * s.y));
    }
};

struct CsrRow {
    __device__ static __forceinline__ int64_t row(const OpCsr &op)
    {
        const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        return i < op.n ? i : -1;
    }
    __device__ static __forceinline__ double2 apply2(const OpCsr &op, int64_t i, const double2 *v,
                                                     double2 vi)
    {
        const int64_t p0 = op.rowptr[i], p1 = op.rowptr[i + 1];
        double sx = 0.0, sy = 0.0;
        int64_t p = p0;
        // four entries at a time: their values and columns, then the four
        // gathered vector elements, are in flight together (rows of the
        // Holstein matrix hold 3 to 5 entries); the sum keeps the entry order
        for (; p + 4 <= p1; p += 4) {
            double2 h[4], x[4];
            int32_t cc[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                h[q] = op.val[p + q];
                cc[q] = op.col[p + q];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) x[q] = v[cc[q]];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                sx = fma(h[q].x, x[q].x, fma(-h[q].y, x[q].y, sx));
                sy = fma(h[q].x, x[q].y, fma(h[q].y, x[q].x, sy));
            }
        }
        for (; p < p1; ++p) {
            const double2 h = op.val[p];
            const double2 x = v[op.col[p]];
            sx = fma(h.x, x.x, fma(-h.y, x.y, sx));
            sy = fma(h.x, x.y, fma(h.y, x.x, sy));
        }
        // (2/a) (H v - b v)
        return make_double2(op.s2 * fma(-op.b, vi.x, sx), op.s2 * fma(-op.b, vi.y, sy));
    }
};

// Matrix-free Holstein states (eq. (ghm)): state i = site * nconf + r.
struct HolRow {
    // state i = site * nconf + r, for i = blockIdx.x * blockDim.x + threadIdx.x:
    // one division per wavefront (the block's first state), then a step or
    // two for threads past a site boundary (n < 2^31: 32-bit arithmetic)
    __device__ static __forceinline__ void split(const OpHol &op, int64_t i, uint32_t &site, uint32_t &r)
    {
        const uint32_t b0 = (uint32_t)(blockIdx.x * blockDim.x);
        uint32_t s = __builtin_amdgcn_readfirstlane(b0 / op.nconf);
        uint32_t rr = (uint32_t)i - s * op.nconf;
        while (rr >= op.nconf) {
            rr -= op.nconf;
            ++s;
        }
        site = s;
        r = rr;
    }
};

// ---------------------------------------------------------------------------
// Host-side construction of the operator parameters from the context
// ---------------------------------------------------------------------------
inline OpChain make_chain(const Ctx &c)
{
    OpChain op;
    op.V = c.V;
    op.dsh = 1.0 / (c.dx * c.dx) - c.b;
    op.s2 = 2.0 / c.a;
    op.off2 = 2.0 * (-0.5 / (c.dx * c.dx)) / c.a;
    op.n = c.n;
    return op;
}

inline OpHoney make_honey(const Ctx &c)
{
    OpHoney op;
    op.eps = c.eps;
    op.b = c.b;
    op.s2 = 2.0 / c.a;
    op.off2 = -2.0 * c.t_hop / c.a;
    op.W = (int32_t)c.W;
    op.L = (int32_t)c.L;
    op.xblocks = (int32_t)((c.L + kBlock - 1) / kBlock);
    op.xcd_remap = 1;
    return op;
}

inline OpHol make_hol(const Ctx &c)
{
    OpHol op;
    op.up = static_cast<const int32_t *>(c.hol_up.p);
    op.dn = static_cast<const int32_t *>(c.hol_dn.p);
    op.occ = static_cast<const uint8_t *>(c.hol_occ.p);
    op.tot = static_cast<const uint8_t *>(c.hol_tot.p);
    const double *site = static_cast<const double *>(c.hol_site.p);
    op.Delta = c.hol_delta ? c.hol_delta : site;
    op.gw0 = site + c.hol_L;
    op.sq = site + 2 * c.hol_L;
    op.w0 = c.hol_w0;
    op.t = c.hol_t;
    op.b = c.b;
    op.s2 = 2.0 / c.a;
    op.L = c.hol_L;
    op.periodic = c.hol_periodic;
    op.n = c.n;
    op.nconf = (uint32_t)c.hol_nconf;
    return op;
}

inline OpCsr make_csr(const Ctx &c)
{
    OpCsr op;
    op.rowptr = c.rowptr;
    op.col = c.col;
    op.val = reinterpret_cast<const double2 *>(c.val);
    op.b = c.b;
    op.s2 = 2.0 / c.a;
    op.n = c.n;
    return op;
}

}  // namespace chebtd
