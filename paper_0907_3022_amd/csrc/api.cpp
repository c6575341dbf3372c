// C ABI of chebtd: context, Hamiltonian builders, bounds, plan, propagation
// and observables.  The time step is the Chebyshev expansion of Sect. 2.2 of
// arXiv:0907.3022; every arithmetic step of it runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>

#include "internal.h"
#include "pair.h"

using namespace chebtd;

struct chebtd_ctx : public Ctx {};

namespace chebtd {
thread_local std::string g_create_err;

int fail(Ctx *c, int code, const std::string &msg)
{
    if (c)
        c->err = msg;
    else
        g_create_err = msg;
    return code;
}

int hip_fail(Ctx *c, hipError_t e, const char *what)
{
    return fail(c, CHEBTD_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

const char *hip_err_name(hipError_t e) { return hipGetErrorName(e); }

void release(DevBuf &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

int ensure(Ctx *c, DevBuf &b, size_t bytes, const char *what)
{
    if (b.bytes >= bytes && b.p) return CHEBTD_OK;
    release(b);
    if (bytes == 0) return CHEBTD_OK;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return fail(c, CHEBTD_E_OOM, std::string("device allocation failed: ") + what + " (" +
                                         std::to_string(bytes) + " bytes)");
    }
    b.bytes = bytes;
    return CHEBTD_OK;
}

void drop_graphs(Ctx *c)
{
    for (auto &g : c->graph_exec) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    for (auto &k : c->graph_key) k = nullptr;
}

// partial-sum buffer big enough for every reduction of the current H
int ensure_partials(Ctx *c)
{
    int64_t nb = (c->n + kBlock - 1) / kBlock;
    nb = std::max<int64_t>(nb, grid_blocks(*c));
    if (pair_supported(*c)) {
        nb = std::max<int64_t>(nb, pair_grid_blocks(*c, c->pair_rows));
        // the head pass writes one partial pair per block
        if (!c->passes.empty() && c->passes[0] > 2)
            nb = std::max<int64_t>(nb, deep_grid_blocks(*c, c->deep_rows[c->passes[0]], c->passes[0]));
    }
    size_t bytes = (size_t)std::max<int64_t>(nb, 1) * 2 * sizeof(double);
    if (c->holstein) {
        size_t hb = (size_t)holstein_obs_blocks(c->hol_nconf) * 3 * c->hol_L * sizeof(double);
        bytes = std::max(bytes, hb);
    }
    return ensure(c, c->partials, bytes, "partials");
}

// Rows per wavefront chunk of the two-orders-per-pass kernel.  Each
// wavefront walks its chunk row by row with one row of loads in flight, so
// short chunks (many wavefronts) hide memory latency best; each chunk also
// re-reads two halo rows of v_k on either side, which costs more once the
// vectors no longer fit the last-level cache.  Measured on MI355X: 2 rows for
// ribbons up to 128 rows wide, 4 below 1024 rows, 16 from there (64M sites).
// CHEBTD_PAIR_ROWS overrides.
int pair_rows_for_width(int64_t W)
{
    const char *env = std::getenv("CHEBTD_PAIR_ROWS");
    if (env) {
        const int r = std::atoi(env);
        if (r >= 1) return r;
    }
    return W <= 128 ? 2 : (W < 1024 ? 4 : 16);
}

int choose_pair_rows(const Ctx &c)
{
    if (c.kind != HKind::Honeycomb) return 1;
    return pair_rows_for_width(c.W);
}

// Lattices of 4M sites and more count as large: the pass costs and chunk
// heights below were measured on MI355X for ribbons of 128x8192 (small),
// 512x32768 and 1024x65536 sites (large).
static bool large_lattice(const Ctx &c) { return c.n >= (int64_t(4) << 20); }

// Rows per wavefront chunk of the D-orders kernel.  Level j of the walk also
// computes D - j halo rows on each side of its chunk, so short chunks repeat
// work and re-read halo rows; large lattices have wavefronts to spare and
// take about 32 rows, small ones 4 to 8 to keep the chip busy.  From 16M
// sites five- and six-order passes take 52 and 56 rows (measured at
// 512x32768: 4.49 against 4.65 ps per site and order for 28 rows, 4.14
// against 4.40 for 32; at 4M sites the taller chunks were 7% slower, too few
// wavefronts).  Below 2^17 sites a pass has only tens of wavefronts, each
// walking its chunk row after row: 4-row chunks at five orders cut a step of
// the 10x1000 and 32x2048 ribbons from 45.7 and 48.7 us to 36.6 and 40.4
// (no change at 64x4096).  Each height makes the walk's rows + 2 (D - 1)
// iterations a whole number of unrolled 6-iteration bodies.
// CHEBTD_DEEP_ROWS overrides.
int choose_deep_rows(const Ctx &c, int D)
{
    if (c.kind != HKind::Honeycomb) return 1;
    if (const char *env = std::getenv("CHEBTD_DEEP_ROWS")) {
        const int r = std::atoi(env);
        if (r >= 1) return r;
    }
    static const int small_rows[kMaxDepth + 1] = {0, 0, 0, 8, 6, 10, 14};
    static const int large_rows[kMaxDepth + 1] = {0, 0, 0, 32, 30, 28, 32};
    static const int huge_rows[kMaxDepth + 1] = {0, 0, 0, 32, 30, 52, 56};
    static const int tiny_rows[kMaxDepth + 1] = {0, 0, 0, 2, 6, 4, 2};
    const bool huge = c.n >= (int64_t(16) << 20), tiny = c.n < (int64_t(1) << 17);
    const int r = (huge ? huge_rows : large_lattice(c) ? large_rows : tiny ? tiny_rows : small_rows)[D];
    return (int)std::min<int64_t>(c.W, r);
}

// Orders per pass for one step of M >= 2 orders on a brick-wall lattice: the
// cheapest split of M into passes of 2 .. kMaxDepth orders and at most one
// single-order pass, by each pass's time relative to a two-order pass
// (measured on MI355X: ribbons as above, a chain of 2^20 sites).  The split
// is fixed by M and the lattice alone, so results never depend on timing.
// CHEBTD_DEPTH=D limits the passes to 1, 2 and D orders (2: pair kernel only).
std::vector<int> plan_passes(const Ctx &c, int M)
{
    static const double small_cost[kMaxDepth + 1] = {0.0, 0.80, 1.0, 1.22, 1.30, 1.26, 1.40};
    static const double large_cost[kMaxDepth + 1] = {0.0, 0.70, 1.0, 1.02, 1.08, 1.00, 1.09};
    static const double chain_cost[kMaxDepth + 1] = {0.0, 0.78, 1.0, 1.27, 2.0, 2.8, 3.6};
    const double *cost = c.kind != HKind::Honeycomb ? chain_cost : large_lattice(c) ? large_cost : small_cost;
    bool allowed[kMaxDepth + 1];
    // the deep kernel addresses the lattice with 32-bit offsets (a chain is
    // one row of n columns)
    const bool chain = c.kind == HKind::Chain;
    const bool deep_ok = deep_offsets_fit(chain ? 1 : c.W, chain ? c.n : c.L);
    for (int d = 0; d <= kMaxDepth; ++d) allowed[d] = d == 1 || d == 2 || (d > 2 && deep_ok);
    if (const char *env = std::getenv("CHEBTD_DEPTH")) {
        const int D = std::max(2, std::min(kMaxDepth, std::atoi(env)));
        for (int d = 3; d <= kMaxDepth; ++d) allowed[d] = d == D && deep_ok;
    }
    // best[m]: cheapest passes for m orders; at most one single-order pass,
    // which only a split of an odd m needs
    std::vector<double> best(M + 1, 1e300);
    std::vector<int> last(M + 1, 0);
    best[0] = 0.0;
    for (int m = 1; m <= M; ++m)
        for (int d = 2; d <= kMaxDepth && d <= m; ++d)
            if (allowed[d] && best[m - d] + cost[d] < best[m]) {
                best[m] = best[m - d] + cost[d];
                last[m] = d;
            }
    // the single-order pass, if any, comes last
    int m = M, tail = 0;
    double total = best[M];
    if (M >= 3 && best[M - 1] + cost[1] < total) {
        m = M - 1;
        tail = 1;
    }
    // every m reached below has a finite cost, hence a last pass of >= 2 orders
    std::vector<int> out;
    for (; m > 0; m -= last[m]) out.push_back(last[m]);
    std::sort(out.begin(), out.end(), [](int x, int y) { return x > y; });
    if (tail) out.push_back(1);
    return out;
}

void invalidate_h(Ctx *c)
{
    c->has_bounds = false;
    c->has_plan = false;
    c->holstein = false;
    drop_graphs(c);
}

void adj_destroy(Ctx *c);    // adjoint.cpp
void batch_destroy(Ctx *c);  // batch.cpp

}  // namespace chebtd

static Ctx *as_ctx(chebtd_ctx *c) { return static_cast<Ctx *>(c); }

extern "C" {

int chebtd_version(void) { return 10000; }

int chebtd_create(chebtd_ctx **out, void *hip_stream)
{
    if (!out) return fail(nullptr, CHEBTD_E_ARG, "chebtd_create: out is null");
    *out = nullptr;
    chebtd_ctx *c = new (std::nothrow) chebtd_ctx();
    if (!c) return fail(nullptr, CHEBTD_E_OOM, "chebtd_create: out of host memory");
    c->stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, c->device);
    if (e == hipSuccess) e = hipMalloc(&c->results.p, 16 * sizeof(double));
    if (e == hipSuccess) {
        c->results.bytes = 16 * sizeof(double);
        e = hipMalloc(&c->counter.p, 4 * sizeof(int64_t));
    }
    if (e == hipSuccess) {
        c->counter.bytes = 4 * sizeof(int64_t);
        e = hipHostMalloc((void **)&c->pinned, 16 * sizeof(double), hipHostMallocDefault);
    }
    if (e == hipSuccess) e = hipEventCreate(&c->ev_a);
    if (e == hipSuccess) e = hipEventCreate(&c->ev_b);
    if (e != hipSuccess) {
        std::string msg = std::string("chebtd_create: ") + hipGetErrorString(e);
        (void)hipGetLastError();
        chebtd_destroy(c);
        return fail(nullptr, CHEBTD_E_HIP, msg);
    }
    *out = c;
    return CHEBTD_OK;
}

int chebtd_destroy(chebtd_ctx *ctx)
{
    if (!ctx) return CHEBTD_OK;
    Ctx *c = as_ctx(ctx);
    (void)hipStreamSynchronize(c->stream);
    adj_destroy(c);
    batch_destroy(c);
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (DevBuf *b : {&c->vA, &c->vB, &c->vC, &c->vD, &c->partials, &c->results, &c->counter, &c->gamma_dev,
                      &c->hol_occ, &c->hol_up, &c->hol_dn,
                      &c->hol_tot, &c->hol_site, &c->hol_binom, &c->chainx})
        release(*b);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->ev_a) (void)hipEventDestroy(c->ev_a);
    if (c->ev_b) (void)hipEventDestroy(c->ev_b);
    delete ctx;
    return CHEBTD_OK;
}

int chebtd_set_stream(chebtd_ctx *ctx, void *hip_stream)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "chebtd_set_stream: null context");
    as_ctx(ctx)->stream = static_cast<hipStream_t>(hip_stream);
    return CHEBTD_OK;
}

const char *chebtd_last_error(const chebtd_ctx *ctx)
{
    if (!ctx) return g_create_err.c_str();
    return static_cast<const Ctx *>(ctx)->err.c_str();
}

int64_t chebtd_dim(const chebtd_ctx *ctx) { return ctx ? static_cast<const Ctx *>(ctx)->n : 0; }

// ---------------------------------------------------------------------------
// builders
// ---------------------------------------------------------------------------
int chebtd_h_chain1d(chebtd_ctx *ctx, int64_t n, double dx, const double *V_dev)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = as_ctx(ctx);
    if (n < 1 || !(dx > 0.0) || !std::isfinite(dx) || !V_dev)
        return fail(c, CHEBTD_E_ARG, "chebtd_h_chain1d: need n >= 1, finite dx > 0, V non-null");
    if (n > ((int64_t)1 << 40)) return fail(c, CHEBTD_E_ARG, "chebtd_h_chain1d: n too large");
    invalidate_h(c);
    c->kind = HKind::Chain;
    c->n = n;
    c->dx = dx;
    c->V = V_dev;
    return ensure_partials(c);
}

int chebtd_h_honeycomb(chebtd_ctx *ctx, int64_t width, int64_t length, int edge, double t_hop,
                       const double *eps_dev)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = as_ctx(ctx);
    if (width < 1 || length < 1 || !eps_dev || !std::isfinite(t_hop) ||
        (edge != CHEBTD_ZIGZAG && edge != CHEBTD_ARMCHAIR))
        return fail(c, CHEBTD_E_ARG,
                    "chebtd_h_honeycomb: need width, length >= 1, a known edge, eps non-null");
    // row and column indices and the block grid are 32-bit in the kernels
    if (width * length >= ((int64_t)1 << 31) || width > 65535 * 4096)
        return fail(c, CHEBTD_E_ARG, "chebtd_h_honeycomb: grid exceeds 2^31 sites");
    invalidate_h(c);
    c->kind = HKind::Honeycomb;
    c->W = width;
    c->L = length;
    c->n = width * length;
    c->edge = edge;
    c->t_hop = t_hop;
    c->eps = eps_dev;
    return ensure_partials(c);
}

int chebtd_h_csr(chebtd_ctx *ctx, int64_t n, int64_t nnz, const int64_t *rowptr_dev,
                 const int32_t *col_dev, const double *val_dev)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = as_ctx(ctx);
    if (n < 1 || nnz < 0 || !rowptr_dev || (nnz > 0 && (!col_dev || !val_dev)))
        return fail(c, CHEBTD_E_ARG, "chebtd_h_csr: need n >= 1, nnz >= 0 and non-null arrays");
    if (n >= (int64_t)INT32_MAX)
        return fail(c, CHEBTD_E_ARG, "chebtd_h_csr: n must fit int32 column indices");
    // reject malformed structure here: the kernels index v with these columns
    int64_t *flag = static_cast<int64_t *>(c->counter.p) + 1;
    hipError_t e = launch_csr_check(c->stream, rowptr_dev, col_dev, n, nnz, flag);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->pinned, flag, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "chebtd_h_csr structure check");
    int64_t bad = 0;
    std::memcpy(&bad, c->pinned, sizeof(int64_t));
    if (bad)
        return fail(c, CHEBTD_E_ARG,
                    "chebtd_h_csr: rowptr must run from 0 to nnz without decreasing and every column "
                    "must lie in [0, n)");
    invalidate_h(c);
    c->kind = HKind::Csr;
    c->n = n;
    c->nnz = nnz;
    c->rowptr = rowptr_dev;
    c->col = col_dev;
    c->val = val_dev;
    return ensure_partials(c);
}

int chebtd_holstein_csr_host(int L, int nph, double t, double w0, const double *g_host,
                             const double *Delta_host, int periodic, int64_t *n_out,
                             int64_t *nnz_out, int64_t *rowptr, int32_t *col, double *val)
{
    HolsteinCsr h;
    std::string err;
    int rc = holstein_build(L, nph, t, w0, g_host, Delta_host, periodic, h, err);
    if (rc) return fail(nullptr, rc, err);
    if (n_out) *n_out = h.n;
    if (nnz_out) *nnz_out = h.nnz;
    if (rowptr) std::memcpy(rowptr, h.rowptr.data(), h.rowptr.size() * sizeof(int64_t));
    if (col) std::memcpy(col, h.col.data(), h.col.size() * sizeof(int32_t));
    if (val) std::memcpy(val, h.val.data(), h.val.size() * sizeof(double));
    return CHEBTD_OK;
}

int chebtd_holstein_occupations(int L, int nph, int64_t *count_out, uint8_t *occ)
{
    if (!count_out) return fail(nullptr, CHEBTD_E_ARG, "count_out is null");
    if (holstein_count(L, nph, count_out)) return fail(nullptr, CHEBTD_E_ARG, "bad L or nph");
    if (!occ) return CHEBTD_OK;
    HolsteinTables h;
    std::string err;
    int rc = holstein_tables(L, nph, 0, h, err);
    if (rc) return fail(nullptr, rc, err);
    // the per-state table is site-major (occ of state site*nconf + r); the
    // export is configuration-major, occ[r*L + j]
    const int64_t C = h.nconf;
    for (int64_t r = 0; r < C; ++r)
        for (int j = 0; j < L; ++j) occ[r * L + j] = h.occ[(size_t)j * (size_t)C + (size_t)r];
    return CHEBTD_OK;
}

int chebtd_h_holstein(chebtd_ctx *ctx, int L, int nph, double t, double w0, const double *g_host,
                      const double *Delta_host, int periodic)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = as_ctx(ctx);
    if (!g_host || !Delta_host || !std::isfinite(t) || !std::isfinite(w0))
        return fail(c, CHEBTD_E_ARG, "chebtd_h_holstein: need g, Delta and finite t, w0");
    for (int i = 0; i < L; ++i)
        if (!std::isfinite(g_host[i]) || !std::isfinite(Delta_host[i]))
            return fail(c, CHEBTD_E_ARG, "chebtd_h_holstein: g and Delta must be finite");
    HolsteinTables h;
    std::string err;
    int rc = holstein_tables(L, nph, periodic, h, err);
    if (rc) return fail(c, rc, err);
    invalidate_h(c);
    c->kind = HKind::None;
    // per-site constants: Delta_i, g_i w0, then sqrt(0 .. nph+1)
    std::vector<double> site((size_t)(2 * L + nph + 2));
    for (int i = 0; i < L; ++i) {
        site[(size_t)i] = Delta_host[i];
        site[(size_t)(L + i)] = g_host[i] * w0;
    }
    for (int q = 0; q <= nph + 1; ++q) site[(size_t)(2 * L + q)] = std::sqrt((double)q);
    if ((rc = ensure(c, c->hol_up, h.up.size() * sizeof(int32_t), "holstein raise table")) ||
        (rc = ensure(c, c->hol_dn, h.dn.size() * sizeof(int32_t), "holstein lower table")) ||
        (rc = ensure(c, c->hol_occ, h.occ.size(), "holstein occupations")) ||
        (rc = ensure(c, c->hol_tot, h.tot.size(), "holstein totals")) ||
        (rc = ensure(c, c->hol_site, site.size() * sizeof(double), "holstein site constants")))
        return rc;
    hipError_t e = hipMemcpy(c->hol_up.p, h.up.data(), h.up.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->hol_dn.p, h.dn.data(), h.dn.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->hol_occ.p, h.occ.data(), h.occ.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->hol_tot.p, h.tot.data(), h.tot.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->hol_site.p, site.data(), site.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(c, e, "chebtd_h_holstein upload");
    c->kind = HKind::Holstein;
    c->n = h.n;
    c->holstein = true;
    c->hol_L = L;
    c->hol_nph = nph;
    c->hol_nconf = h.nconf;
    c->hol_t = t;
    c->hol_w0 = w0;
    c->hol_periodic = periodic ? 1 : 0;
    // binomials C(a, m), a <= nph + L + 1, m <= L, for the walk's own partner
    // ranks.  The entries it reads are at most C(nph + L, L) = nconf and
    // C(nph + L, L - 1) = nconf L / (nph + 1), both below the dimension
    // L nconf < 2^31; the last row may exceed 2^31 and is stored saturated.
    // The walk ranks the partners itself where the tables would stream from
    // HBM (measured on MI355X: the L = 18 polaron, 6.2e8 states, 10.6 -> 9.4
    // ms per order), and reads the tables where the last-level cache holds
    // them (the L = 10 ring, 1.85M states: 23.2 us against 30.8 us ranking);
    // CHEBTD_HOL_RANK=1 or 0 forces either
    c->hol_brows = 0;
    {
        const int brows = nph + L + 2, bcols = L + 1;
        const char *renv = std::getenv("CHEBTD_HOL_RANK");
        const bool want = renv ? std::atoi(renv) != 0 : h.n > ((int64_t)8 << 20);
        if (want && (size_t)brows * bcols * sizeof(int32_t) <= (size_t)kHolBinomBytes) {
            // Pascal's rule in 64 bits, stored saturated at INT32_MAX
            std::vector<int64_t> c64((size_t)brows * bcols, 0);
            std::vector<int32_t> cb((size_t)brows * bcols, 0);
            for (int a = 0; a < brows; ++a) {
                c64[(size_t)a * bcols] = 1;
                for (int m = 1; m <= std::min(a, L); ++m)
                    c64[(size_t)a * bcols + m] = std::min<int64_t>(
                        c64[(size_t)(a - 1) * bcols + m - 1] + (m <= a - 1 ? c64[(size_t)(a - 1) * bcols + m] : 0),
                        INT32_MAX);
            }
            for (size_t q = 0; q < cb.size(); ++q) cb[q] = (int32_t)c64[q];
            if ((rc = ensure(c, c->hol_binom, cb.size() * sizeof(int32_t), "holstein binomials"))) return rc;
            e = hipMemcpy(c->hol_binom.p, cb.data(), cb.size() * sizeof(int32_t), hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_fail(c, e, "chebtd_h_holstein binomials");
            c->hol_brows = brows;
        }
    }
    // tuning and test override: electron sites per thread of the order walk
    // (0: all L sites per thread)
    c->hol_spt = 0;
    if (const char *env = std::getenv("CHEBTD_HOL_SPT")) c->hol_spt = std::max(0, std::atoi(env));
    // XCD-contiguous block order for the walk (measured on MI355X at the
    // polaron size: 14.6 -> 13.6 ms per order); CHEBTD_HOL_REMAP=0 turns it off
    c->hol_remap = 1;
    if (const char *env = std::getenv("CHEBTD_HOL_REMAP")) c->hol_remap = std::atoi(env) ? 1 : 0;
    return ensure_partials(c);
}

// ---------------------------------------------------------------------------
// bounds and plan
// ---------------------------------------------------------------------------
int chebtd_gershgorin(chebtd_ctx *ctx, double *emin, double *emax)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = as_ctx(ctx);
    if (!emin || !emax) return fail(c, CHEBTD_E_ARG, "chebtd_gershgorin: null output");
    if (c->kind == HKind::None) return fail(c, CHEBTD_E_STATE, "chebtd_gershgorin: no Hamiltonian");
    double *res = static_cast<double *>(c->results.p);
    hipError_t e = launch_gershgorin(*c, c->stream, static_cast<double *>(c->partials.p), res);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->pinned, res, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "chebtd_gershgorin");
    *emin = c->pinned[0];
    *emax = c->pinned[1];
    return CHEBTD_OK;
}

int chebtd_set_bounds(chebtd_ctx *ctx, double emin, double emax, double alpha)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = as_ctx(ctx);
    if (!(emax > emin) || !std::isfinite(emin) || !std::isfinite(emax) || !(alpha >= 0.0) ||
        !std::isfinite(alpha))
        return fail(c, CHEBTD_E_ARG, "chebtd_set_bounds: need finite emax > emin and alpha >= 0");
    c->emin = emin;
    c->emax = emax;
    c->alpha = alpha;
    shift_scale(emin, emax, alpha, &c->a, &c->b);
    c->has_bounds = true;
    c->has_plan = false;
    drop_graphs(c);
    return CHEBTD_OK;
}

static int plan_common(Ctx *c, double dt, int M)
{
    step_weights(c->a, c->b, dt, M, c->gamma);
    int rc;
    if ((rc = ensure(c, c->gamma_dev, c->gamma.size() * sizeof(double), "weights"))) return rc;
    hipError_t e = hipMemcpy(c->gamma_dev.p, c->gamma.data(), c->gamma.size() * sizeof(double),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(c, e, "chebtd_plan upload");
    const size_t vbytes = (size_t)c->n * 2 * sizeof(double);
    if ((rc = ensure(c, c->vA, vbytes, "work vector A")) || (rc = ensure(c, c->vB, vbytes, "work vector B")))
        return rc;
    // two more vectors let brick-wall Hamiltonians advance two orders per pass
    c->use_pairs = false;
    c->passes.clear();
    c->pair_rows = choose_pair_rows(*c);
    if (pair_supported(*c) && M >= 2) {
        if ((rc = ensure(c, c->vC, vbytes, "work vector C")) || (rc = ensure(c, c->vD, vbytes, "work vector D")))
            return rc;
        c->use_pairs = true;
        c->passes = plan_passes(*c, M);
        for (int d = 3; d <= kMaxDepth; ++d) c->deep_rows[d] = choose_deep_rows(*c, d);
    }
    if ((rc = ensure_partials(c))) return rc;
    if (c->kind == HKind::Chain) {
        const size_t xb = chain_multi_scratch_bytes(chain_multi_config(c->n));
        if (xb && (rc = ensure(c, c->chainx, xb, "chain exchange scratch"))) return rc;
    }
    c->dt = dt;
    c->M = M;
    c->has_plan = true;
    c->plan_version++;
    drop_graphs(c);
    return CHEBTD_OK;
}

int chebtd_plan(chebtd_ctx *ctx, double dt, double tol, int *M_out)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = as_ctx(ctx);
    if (c->kind == HKind::None) return fail(c, CHEBTD_E_STATE, "chebtd_plan: no Hamiltonian");
    if (!c->has_bounds) return fail(c, CHEBTD_E_STATE, "chebtd_plan: set the spectral bounds first");
    if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(c, CHEBTD_E_ARG, "chebtd_plan: need finite dt >= 0");
    if (!(tol > 0.0)) tol = 1e-15;
    const int M = truncation_order(c->a * dt, tol);
    if (M < 0) return fail(c, CHEBTD_E_ARG, "chebtd_plan: bad a*dt or tol");
    int rc = plan_common(c, dt, M);
    if (rc) return rc;
    if (M_out) *M_out = M;
    return CHEBTD_OK;
}

int chebtd_plan_order(chebtd_ctx *ctx, double dt, int M)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = as_ctx(ctx);
    if (c->kind == HKind::None) return fail(c, CHEBTD_E_STATE, "chebtd_plan_order: no Hamiltonian");
    if (!c->has_bounds) return fail(c, CHEBTD_E_STATE, "chebtd_plan_order: set bounds first");
    if (!(dt >= 0.0) || !std::isfinite(dt) || M < 0 || M > 10000000)
        return fail(c, CHEBTD_E_ARG, "chebtd_plan_order: need dt >= 0 and 0 <= M <= 1e7");
    return plan_common(c, dt, M);
}

int chebtd_get_plan(const chebtd_ctx *ctx, double *gamma_host, double *a, double *b, double *dt,
                    int *M)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    const Ctx *c = static_cast<const Ctx *>(ctx);
    if (!c->has_plan) return fail(const_cast<Ctx *>(c), CHEBTD_E_STATE, "chebtd_get_plan: no plan");
    if (gamma_host) std::memcpy(gamma_host, c->gamma.data(), c->gamma.size() * sizeof(double));
    if (a) *a = c->a;
    if (b) *b = c->b;
    if (dt) *dt = c->dt;
    if (M) *M = c->M;
    return CHEBTD_OK;
}

int chebtd_plan_passes(const chebtd_ctx *ctx, int *passes_out, int capacity, int *count_out)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    const Ctx *c = static_cast<const Ctx *>(ctx);
    if (!c->has_plan) return fail(const_cast<Ctx *>(c), CHEBTD_E_STATE, "chebtd_plan_passes: no plan");
    if (capacity < 0 || (capacity > 0 && !passes_out))
        return fail(const_cast<Ctx *>(c), CHEBTD_E_ARG, "chebtd_plan_passes: bad output array");
    const int n = c->use_pairs ? (int)c->passes.size() : 0;
    for (int i = 0; i < n && i < capacity; ++i) passes_out[i] = c->passes[i];
    if (count_out) *count_out = n;
    return CHEBTD_OK;
}

int chebtd_set_check_tol(chebtd_ctx *ctx, double rel_tol)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    if (!(rel_tol > 0.0)) return fail(as_ctx(ctx), CHEBTD_E_ARG, "check tolerance must be > 0");
    as_ctx(ctx)->check_tol = rel_tol;
    return CHEBTD_OK;
}

}  // extern "C"
