// Time stepping and observables of chebtd (Sect. 2.2 and Sect. 3 of
// arXiv:0907.3022).  One step: the head kernel forms v_1 = H~ psi and
// acc = gamma_0 psi + gamma_1 v_1, then M-1 fused recursion kernels form
// v_{k+1} = 2 H~ v_k - v_{k-1} and acc += gamma_{k+1} v_{k+1}; acc is the
// next state.  Buffers rotate so that no copy is made inside the K steps.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "internal.h"
#include "pair.h"

namespace chebtd {
int fail(Ctx *c, int code, const std::string &msg);
int hip_fail(Ctx *c, hipError_t e, const char *what);
int ensure(Ctx *c, DevBuf &b, size_t bytes, const char *what);
void release(DevBuf &b);
void drop_graphs(Ctx *c);
bool adj_begin_run(Ctx *c, int64_t K);                         // adjoint.cpp
double2 *adj_checkpoint(Ctx *c, int64_t step, int64_t K);  // adjoint.cpp
double2 *adj_step_ends(Ctx *c, int64_t step);              // adjoint.cpp
}  // namespace chebtd

using namespace chebtd;
struct chebtd_ctx : public Ctx {};

namespace {

double2 weight(const Ctx *c, int k)
{
    if (k > c->M) return make_double2(0.0, 0.0);
    return make_double2(c->gamma[2 * (size_t)k], c->gamma[2 * (size_t)k + 1]);
}

// Orders of the multi-order pass a step runs most often after its head (ties:
// the deeper), or the head's own when no such pass follows it.
int dominant_pass(const Ctx &c)
{
    int count[kMaxDepth + 1] = {};
    for (size_t i = 1; i < c.passes.size(); ++i)
        if (c.passes[i] >= 2) ++count[c.passes[i]];
    int best = c.passes.empty() ? 2 : c.passes[0];
    int most = 0;
    for (int d = 2; d <= kMaxDepth; ++d)
        if (count[d] > 0 && count[d] >= most) {
            most = count[d];
            best = d;
        }
    return best;
}

// One time step with several orders per pass (brick-wall H, M >= 2), in the
// passes the plan chose: the head pass forms v_1 .. v_D and starts acc; each
// further pass forms its orders from the previous two vectors (2 orders: the
// pair kernel, 3 .. kMaxDepth: the deep kernel); a single-order pass, if
// any, comes last.  Pass outputs alternate between (vA, vC) and (vD, cur):
// cur is free once the head pass has read it.
// ends (or null): 2 n values that receive v_{M-1}, v_M of the step
hipError_t enqueue_step_pairs(Ctx *c, hipStream_t s, double2 *cur, double2 *nxt, double2 *ckpt, double2 *ends,
                              double *norm_out, double *energy_out)
{
    double2 *A = static_cast<double2 *>(c->vA.p), *C = static_cast<double2 *>(c->vC.p),
            *D = static_cast<double2 *>(c->vD.p);
    double *partials = static_cast<double *>(c->partials.p);
    const std::vector<int> &P = c->passes;
    const int h = P[0];
    double2 g[kMaxDepth + 1];
    hipError_t e;
    int64_t nhead;  // blocks of the head pass (one partial pair each)
    // the last multi-order pass writes its two orders, v_{M-1} and v_M, into
    // ends; without ends nothing reads them (the next step starts from acc),
    // so a deep last pass writes acc alone (32 of its 104 B per site fewer)
    const bool head_last = P.size() == 1;
    double2 *h1 = ends && head_last ? ends : A, *h2 = ends && head_last ? ends + c->n : C;
    if (head_last && !ends && h > 2) h1 = h2 = nullptr;
    if (h > 2) {
        for (int j = 0; j <= h; ++j) g[j] = weight(c, j);
        e = launch_deep(*c, s, h, c->deep_rows[h], true, nullptr, cur, h1, h2, nxt, g, ckpt, partials, nullptr);
        nhead = deep_grid_blocks(*c, c->deep_rows[h], h);
    } else {
        e = launch_pair(*c, s, c->pair_rows, true, nullptr, cur, h1, h2, nxt, weight(c, 0), weight(c, 1),
                        weight(c, 2), ckpt, partials);
        nhead = pair_grid_blocks(*c, c->pair_rows);
    }
    if (e != hipSuccess) return e;
    // the step's norm and energy: finished by block 0 of the next multi-order
    // pass when there is one (no extra launch), else by their own kernel
    const NeFinal fin{partials, (int)nhead, c->a, c->b, norm_out, energy_out,
                      static_cast<int64_t *>(c->counter.p)};
    const bool want_ne = norm_out || energy_out;
    const bool has_next = P.size() > 1 && P[1] >= 2;
    if (want_ne && !has_next) {
        e = launch_finalize_ne(s, partials, fin.nparts, c->a, c->b, norm_out, energy_out, fin.counter, nullptr);
        if (e != hipSuccess) return e;
    }
    double2 *X = A, *Y = C, *F1 = D, *F2 = cur;  // (v_{k-1}, v_k) and the free pair
    int k = h;
    for (size_t i = 1; i < P.size(); ++i) {
        const int d = P[i];
        const NeFinal *f = (want_ne && i == 1) ? &fin : nullptr;
        if (ends && i + 1 == P.size() && d >= 2) {
            F1 = ends;
            F2 = ends + c->n;
        }
        if (d == 1) {  // the last order: v_M = 2 H~ v_{M-1} - v_{M-2} over v_{M-2}
            e = launch_iter(*c, s, Y, X, nxt, weight(c, k + 1));
            if (e == hipSuccess && ends) e = launch_copy(s, Y, ends, c->n);
            if (e == hipSuccess && ends) e = launch_copy(s, X, ends + c->n, c->n);
        } else if (d == 2) {
            e = launch_pair(*c, s, c->pair_rows, false, X, Y, F1, F2, nxt, make_double2(0.0, 0.0),
                            weight(c, k + 1), weight(c, k + 2), nullptr, nullptr, f);
        } else {
            g[0] = make_double2(0.0, 0.0);
            for (int j = 1; j <= d; ++j) g[j] = weight(c, k + j);
            const bool last = i + 1 == P.size() && !ends;
            e = launch_deep(*c, s, d, c->deep_rows[d], false, X, Y, last ? nullptr : F1, last ? nullptr : F2, nxt,
                            g, nullptr, nullptr, f);
        }
        if (e != hipSuccess) return e;
        k += d;
        double2 *t1 = X, *t2 = Y;
        X = F1;
        Y = F2;
        F1 = t1;
        F2 = t2;
    }
    return k == c->M ? hipSuccess : hipErrorInvalidValue;
}

// Enqueue one time step: cur -> nxt.  cur is overwritten with v_2, v_4, ...
hipError_t enqueue_step(Ctx *c, hipStream_t s, double2 *cur, double2 *nxt, double2 *ckpt, double2 *ends,
                        double *norm_out, double *energy_out, unsigned flags)
{
    if (c->use_pairs && !(flags & CHEBTD_SINGLE_ORDER))
        return enqueue_step_pairs(c, s, cur, nxt, ckpt, ends, norm_out, energy_out);
    double2 *A = static_cast<double2 *>(c->vA.p);
    double *partials = static_cast<double *>(c->partials.p);
    hipError_t e = launch_head(*c, s, cur, A, nxt, weight(c, 0), weight(c, 1), ckpt, partials);
    if (e != hipSuccess) return e;
    if (norm_out || energy_out) {
        e = launch_finalize_ne(s, partials, (int)head_blocks(*c), c->a, c->b, norm_out, energy_out,
                               static_cast<int64_t *>(c->counter.p), nullptr);
        if (e != hipSuccess) return e;
    }
    // the Holstein and CSR operators add the weighted orders to acc every
    // third order and at the step's last (acc holds orders 0 .. done); the
    // stencils every order
    int done = 1;
    const bool lazy = c->kind == HKind::Holstein || c->kind == HKind::Csr;
    for (int k = 1; k <= c->M - 1; ++k) {
        double2 *vk = (k & 1) ? A : cur;
        double2 *vprev = (k & 1) ? cur : A;
        if (lazy) {
            const int pend = k + 1 - done;  // orders done+1 .. k+1 not yet in acc
            const int nacc = (pend == 3 || k + 1 == c->M) ? pend : 0;
            e = launch_iter_lazy(*c, s, vk, vprev, nxt, nacc, weight(c, k - 1), weight(c, k), weight(c, k + 1));
            if (nacc) done = k + 1;
        } else {
            e = launch_iter(*c, s, vk, vprev, nxt, weight(c, k + 1));
        }
        if (e != hipSuccess) return e;
    }
    if (ends && c->M >= 1) {
        // v_M was written over v_{M-2}: A holds the odd orders, cur the even ones
        double2 *vM = (c->M & 1) ? A : cur, *vM1 = (c->M & 1) ? cur : A;
        e = launch_copy(s, vM1, ends, c->n);
        if (e == hipSuccess) e = launch_copy(s, vM, ends + c->n, c->n);
    }
    return e;
}

// norm of psi into results[slot]
hipError_t enqueue_norm(Ctx *c, hipStream_t s, const double2 *psi, int slot)
{
    double *partials = static_cast<double *>(c->partials.p);
    hipError_t e = launch_norm(*c, s, psi, partials);
    if (e != hipSuccess) return e;
    return launch_sum_partials(s, partials, (int)reduce_blocks(c->n), 2,
                               static_cast<double *>(c->results.p) + slot);
}

// Two steps (psi -> B -> psi) captured once into a graph and replayed.
int get_pair_graph(Ctx *c, double2 *psi, double *norm_out, double *energy_out, unsigned flags,
                   hipGraphExec_t *out)
{
    const void *key[4] = {psi, norm_out, energy_out,
                          reinterpret_cast<const void *>((uintptr_t)(flags & CHEBTD_SINGLE_ORDER) + 1)};
    if (c->graph_exec[0] && key[0] == c->graph_key[0] && key[1] == c->graph_key[1] &&
        key[2] == c->graph_key[2] && key[3] == c->graph_key[3]) {
        *out = c->graph_exec[0];
        return CHEBTD_OK;
    }
    drop_graphs(c);
    hipError_t e = hipSuccess;
    if (!c->cap_stream) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(c, e, "graph stream");
    double2 *B = static_cast<double2 *>(c->vB.p);
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamBeginCapture");
    hipError_t e1 = enqueue_step(c, c->cap_stream, psi, B, nullptr, nullptr, norm_out, energy_out, flags);
    hipError_t e2 = e1 == hipSuccess ? enqueue_step(c, c->cap_stream, B, psi, nullptr, nullptr, norm_out, energy_out, flags)
                                     : e1;
    e = hipStreamEndCapture(c->cap_stream, &g);
    if (e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(c, e2, "graph capture of a step");
    }
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&c->graph_exec[0], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->graph_exec[0] = nullptr;
        return hip_fail(c, e, "hipGraphInstantiate");
    }
    for (int i = 0; i < 4; ++i) c->graph_key[i] = key[i];
    *out = c->graph_exec[0];
    return CHEBTD_OK;
}

}  // namespace

extern "C" {

int chebtd_propagate(chebtd_ctx *ctx, double *psi_dev, int64_t K, double *norm_dev,
                     double *energy_dev, unsigned flags)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = static_cast<Ctx *>(ctx);
    if (!c->has_plan) return fail(c, CHEBTD_E_STATE, "chebtd_propagate: no plan");
    if (!psi_dev || K < 0) return fail(c, CHEBTD_E_ARG, "chebtd_propagate: need psi and K >= 0");
    const bool keep = (flags & CHEBTD_KEEP_CHECKPOINTS) != 0;
    // a checkpointing run of zero steps is a run too (its adjoint is the
    // identity), so that no earlier trajectory stays current after it
    if (keep && !adj_begin_run(c, K))
        return fail(c, CHEBTD_E_STATE,
                    "chebtd_propagate: checkpoints need chebtd_reserve_adjoint with max_steps >= K");
    if (K == 0) return CHEBTD_OK;
    const bool check = (flags & CHEBTD_NO_CHECK) == 0;
    hipStream_t s = c->stream;
    double2 *P = reinterpret_cast<double2 *>(psi_dev);
    double2 *B = static_cast<double2 *>(c->vB.p);
    hipError_t e = hipSuccess;

    if (check) {
        e = enqueue_norm(c, s, P, 0);
        if (e != hipSuccess) return hip_fail(c, e, "initial norm");
    }
    if (norm_dev || energy_dev) {
        e = launch_reset_counter(s, static_cast<int64_t *>(c->counter.p));
        if (e != hipSuccess) return hip_fail(c, e, "counter reset");
    }

    // the one-workgroup chain kernel keeps psi_s but not the step-end pairs
    const bool small = c->kind == HKind::Chain && chain_small_fits(c->n) &&
                       !(flags & CHEBTD_NO_PERSISTENT) && !(keep && adj_step_ends(c, 0));
    if (small) {
        e = launch_chain_small(*c, s, P, P, static_cast<const double2 *>(c->gamma_dev.p), K, norm_dev,
                               energy_dev, keep ? adj_checkpoint(c, 0, K) : nullptr);
        if (e != hipSuccess) return hip_fail(c, e, "persistent chain kernel");
    } else if ((flags & CHEBTD_GRAPH) && !keep) {
        hipGraphExec_t ge = nullptr;
        int rc = get_pair_graph(c, P, norm_dev, energy_dev, flags, &ge);
        if (rc) return rc;
        for (int64_t s2 = 0; s2 + 1 < K; s2 += 2) {
            e = hipGraphLaunch(ge, s);
            if (e != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
        }
        if (K & 1) {
            e = enqueue_step(c, s, P, B, nullptr, nullptr, norm_dev, energy_dev, flags);
            if (e == hipSuccess) e = launch_copy(s, B, P, c->n);
            if (e != hipSuccess) return hip_fail(c, e, "last step");
        }
    } else {
        for (int64_t st = 0; st < K; ++st) {
            double2 *cur = (st & 1) ? B : P;
            double2 *nxt = (st & 1) ? P : B;
            e = enqueue_step(c, s, cur, nxt, keep ? adj_checkpoint(c, st, K) : nullptr,
                             keep ? adj_step_ends(c, st) : nullptr, norm_dev, energy_dev, flags);
            if (e != hipSuccess) return hip_fail(c, e, "step launch");
        }
        if (K & 1) {
            e = launch_copy(s, B, P, c->n);
            if (e != hipSuccess) return hip_fail(c, e, "final copy");
        }
    }

    if (!check) return CHEBTD_OK;
    e = enqueue_norm(c, s, P, 2);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->pinned, c->results.p, 4 * sizeof(double), hipMemcpyDeviceToHost, s);
    // the several-workgroup chain run's wait limit
    int32_t *tflag = small ? chain_multi_timeout(*c) : nullptr;
    if (e == hipSuccess && tflag) e = hipMemcpyAsync(c->pinned + 8, tflag, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "norm check");
    if (tflag) {
        int32_t timed_out = 0;
        std::memcpy(&timed_out, c->pinned + 8, sizeof(int32_t));
        if (timed_out)
            return fail(c, CHEBTD_E_TIMEOUT,
                        "chebtd_propagate: a chain workgroup's wait for its neighbours ran out; psi is invalid");
    }
    const double n0 = c->pinned[0], n1 = c->pinned[2];
    if (!std::isfinite(n1) || !std::isfinite(n0) || std::fabs(n1 - n0) > c->check_tol * n0) {
        return fail(c, CHEBTD_E_DIVERGED,
                    "chebtd_propagate: norm went from " + std::to_string(n0) + " to " +
                        std::to_string(n1) + "; the spectral bounds do not enclose H");
    }
    return CHEBTD_OK;
}

int chebtd_propagate_td(chebtd_ctx *ctx, double *psi_dev, int64_t K, const double *onsite_dev,
                        int64_t stride, double *norm_dev, double *energy_dev, unsigned flags)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = static_cast<Ctx *>(ctx);
    if (!c->has_plan) return fail(c, CHEBTD_E_STATE, "chebtd_propagate_td: no plan");
    if (!psi_dev || K < 0 || !onsite_dev)
        return fail(c, CHEBTD_E_ARG, "chebtd_propagate_td: need psi, K >= 0 and the on-site schedule");
    if (flags & CHEBTD_KEEP_CHECKPOINTS)
        return fail(c, CHEBTD_E_ARG, "chebtd_propagate_td: checkpoints are not kept for a time-dependent H");
    const int64_t need = c->kind == HKind::Holstein ? c->hol_L : c->n;
    if (c->kind != HKind::Chain && c->kind != HKind::Honeycomb && c->kind != HKind::Holstein)
        return fail(c, CHEBTD_E_STATE, "chebtd_propagate_td: needs a chain, ribbon or Holstein H");
    if (stride < need) return fail(c, CHEBTD_E_ARG, "chebtd_propagate_td: stride smaller than one step's values");
    if (K == 0) return CHEBTD_OK;
    // one launch sequence per step with that step's on-site values; the
    // borrowed pointer is restored afterwards
    const double *saved = c->kind == HKind::Chain ? c->V : c->eps;
    const unsigned step_flags = (flags & ~(CHEBTD_GRAPH)) | CHEBTD_NO_PERSISTENT;
    hipStream_t s = c->stream;
    double2 *P = reinterpret_cast<double2 *>(psi_dev);
    double2 *B = static_cast<double2 *>(c->vB.p);
    hipError_t e = hipSuccess;
    const bool check = (flags & CHEBTD_NO_CHECK) == 0;
    if (check) e = enqueue_norm(c, s, P, 0);
    if (e == hipSuccess && (norm_dev || energy_dev)) e = launch_reset_counter(s, static_cast<int64_t *>(c->counter.p));
    for (int64_t st = 0; st < K && e == hipSuccess; ++st) {
        const double *on = onsite_dev + st * stride;
        if (c->kind == HKind::Chain)
            c->V = on;
        else if (c->kind == HKind::Honeycomb)
            c->eps = on;
        else
            c->hol_delta = on;
        double2 *cur = (st & 1) ? B : P;
        double2 *nxt = (st & 1) ? P : B;
        e = enqueue_step(c, s, cur, nxt, nullptr, nullptr, norm_dev, energy_dev, step_flags);
    }
    if (c->kind == HKind::Chain)
        c->V = saved;
    else if (c->kind == HKind::Honeycomb)
        c->eps = saved;
    c->hol_delta = nullptr;
    if (e == hipSuccess && (K & 1)) e = launch_copy(s, B, P, c->n);
    if (e != hipSuccess) return hip_fail(c, e, "chebtd_propagate_td");
    if (!check) return CHEBTD_OK;
    e = enqueue_norm(c, s, P, 2);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->pinned, c->results.p, 4 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "norm check");
    const double n0 = c->pinned[0], n1 = c->pinned[2];
    if (!std::isfinite(n1) || !std::isfinite(n0) || std::fabs(n1 - n0) > c->check_tol * n0)
        return fail(c, CHEBTD_E_DIVERGED,
                    "chebtd_propagate_td: norm went from " + std::to_string(n0) + " to " + std::to_string(n1) +
                        "; the bounds do not enclose every step's H");
    return CHEBTD_OK;
}

int chebtd_density(chebtd_ctx *ctx, const double *psi_dev, double *rho_dev)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = static_cast<Ctx *>(ctx);
    if (c->kind == HKind::None) return fail(c, CHEBTD_E_STATE, "chebtd_density: no Hamiltonian");
    if (!psi_dev || !rho_dev) return fail(c, CHEBTD_E_ARG, "chebtd_density: null pointer");
    hipError_t e = launch_density(c->stream, reinterpret_cast<const double2 *>(psi_dev), rho_dev, c->n);
    return e == hipSuccess ? CHEBTD_OK : hip_fail(c, e, "chebtd_density");
}

int chebtd_region_sum(chebtd_ctx *ctx, const double *psi_dev, const uint8_t *mask_dev,
                      double *out_dev)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = static_cast<Ctx *>(ctx);
    if (c->kind == HKind::None) return fail(c, CHEBTD_E_STATE, "chebtd_region_sum: no Hamiltonian");
    if (!psi_dev || !mask_dev || !out_dev) return fail(c, CHEBTD_E_ARG, "chebtd_region_sum: null pointer");
    // out_dev receives the sum; partials go to the context's scratch
    double *res = static_cast<double *>(c->results.p) + 8;
    hipError_t e = launch_region(c->stream, reinterpret_cast<const double2 *>(psi_dev), mask_dev, c->n,
                                 static_cast<double *>(c->partials.p), res);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out_dev, res, sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    return e == hipSuccess ? CHEBTD_OK : hip_fail(c, e, "chebtd_region_sum");
}

int chebtd_norm_energy(chebtd_ctx *ctx, const double *psi_dev, double *out2_dev)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = static_cast<Ctx *>(ctx);
    if (c->kind == HKind::None || !c->has_bounds)
        return fail(c, CHEBTD_E_STATE, "chebtd_norm_energy: needs a Hamiltonian and bounds");
    if (!psi_dev || !out2_dev) return fail(c, CHEBTD_E_ARG, "chebtd_norm_energy: null pointer");
    double *partials = static_cast<double *>(c->partials.p);
    hipError_t e = launch_head(*c, c->stream, reinterpret_cast<const double2 *>(psi_dev), nullptr,
                               nullptr, make_double2(0, 0), make_double2(0, 0), nullptr, partials);
    if (e == hipSuccess)
        e = launch_finalize_ne(c->stream, partials, (int)head_blocks(*c), c->a, c->b, nullptr, nullptr,
                               nullptr, out2_dev);
    return e == hipSuccess ? CHEBTD_OK : hip_fail(c, e, "chebtd_norm_energy");
}

int chebtd_holstein_obs(chebtd_ctx *ctx, const double *psi_dev, double *n_dev, double *nph_dev,
                        double *chi_dev)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = static_cast<Ctx *>(ctx);
    if (!c->holstein) return fail(c, CHEBTD_E_STATE, "chebtd_holstein_obs: H is not a Holstein model");
    if (!psi_dev || !n_dev || !nph_dev || !chi_dev)
        return fail(c, CHEBTD_E_ARG, "chebtd_holstein_obs: null pointer");
    hipError_t e = launch_holstein_obs(
        c->stream, reinterpret_cast<const double2 *>(psi_dev), static_cast<const uint8_t *>(c->hol_occ.p),
        static_cast<const int32_t *>(c->hol_up.p), c->hol_nconf, c->hol_L,
        static_cast<double *>(c->partials.p), n_dev, nph_dev, chi_dev);
    return e == hipSuccess ? CHEBTD_OK : hip_fail(c, e, "chebtd_holstein_obs");
}

int chebtd_time_recursion_kernel(chebtd_ctx *ctx, int launches, unsigned flags, double *ms_per_launch,
                                 const char **name_out, int *orders_out)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = static_cast<Ctx *>(ctx);
    if (!c->has_plan) return fail(c, CHEBTD_E_STATE, "chebtd_time_recursion_kernel: no plan");
    if (launches < 1 || !ms_per_launch) return fail(c, CHEBTD_E_ARG, "need launches >= 1 and an output");
    const bool pairs = c->use_pairs && !(flags & CHEBTD_SINGLE_ORDER);
    // the multi-order kernel the step spends most of its passes in
    const int dp = pairs ? dominant_pass(*c) : 2;
    static const char *names[] = {"k_iter_chain", "k_iter_honey<0>", "k_iter_honey<1>", "k_iter_csr",
                                  "k_pair<0,false>", "k_pair<1,false>", "k_iter_hol<true, false>", "k_iter_hol<false, false>"};
    // [edge][streaming stores][orders per pass]
    static const char *deep_names[2][2][kMaxDepth + 1] = {
        {{"", "", "", "k_deep<0,3,false,false>", "k_deep<0,4,false,false>", "k_deep<0,5,false,false>",
          "k_deep<0,6,false,false>"},
         {"", "", "", "k_deep<0,3,false,true>", "k_deep<0,4,false,true>", "k_deep<0,5,false,true>",
          "k_deep<0,6,false,true>"}},
        {{"", "", "", "k_deep<1,3,false,false>", "k_deep<1,4,false,false>", "k_deep<1,5,false,false>",
          "k_deep<1,6,false,false>"},
         {"", "", "", "k_deep<1,3,false,true>", "k_deep<1,4,false,true>", "k_deep<1,5,false,true>",
          "k_deep<1,6,false,true>"}}};
    const bool arm = c->kind == HKind::Honeycomb && c->edge == CHEBTD_ARMCHAIR;
    const char *nm = (pairs && dp > 2) ? deep_names[arm ? 1 : 0][deep_stream_stores(*c) ? 1 : 0][dp]
                     : pairs ? (arm ? names[5] : names[4])
                     : c->kind == HKind::Chain    ? names[0]
                     : c->kind == HKind::Csr      ? names[3]
                     : c->kind == HKind::Holstein ? names[c->hol_brows > 0 ? 6 : 7]
                     : (c->edge == CHEBTD_ZIGZAG ? names[1] : names[2]);
    if (name_out) *name_out = nm;
    if (orders_out) *orders_out = pairs ? dp : 1;
    // scratch: four vectors and an accumulator, zeroed
    DevBuf scratch;
    const size_t vb = (size_t)c->n * sizeof(double2);
    int rc = ensure(c, scratch, 5 * vb, "timing vectors");
    if (rc) return rc;
    hipStream_t s = c->stream;
    double2 *V0 = static_cast<double2 *>(scratch.p), *V1 = V0 + c->n, *V2 = V1 + c->n, *V3 = V2 + c->n,
            *acc = V3 + c->n;
    hipError_t e = hipMemsetAsync(scratch.p, 0, 5 * vb, s);
    double2 gd[kMaxDepth + 1];
    for (int j = 0; j <= dp; ++j) gd[j] = weight(c, j < 1 ? 1 : j);
    gd[0] = make_double2(0.0, 0.0);
    auto one = [&](int i) -> hipError_t {
        if (pairs && dp > 2)
            return (i & 1) ? launch_deep(*c, s, dp, c->deep_rows[dp], false, V2, V3, V0, V1, acc, gd, nullptr,
                                         nullptr, nullptr)
                           : launch_deep(*c, s, dp, c->deep_rows[dp], false, V0, V1, V2, V3, acc, gd, nullptr,
                                         nullptr, nullptr);
        if (pairs)
            return (i & 1) ? launch_pair(*c, s, c->pair_rows, false, V2, V3, V0, V1, acc, make_double2(0, 0),
                                         weight(c, 1), weight(c, 2), nullptr, nullptr)
                           : launch_pair(*c, s, c->pair_rows, false, V0, V1, V2, V3, acc, make_double2(0, 0),
                                         weight(c, 1), weight(c, 2), nullptr, nullptr);
        if (c->kind == HKind::Holstein || c->kind == HKind::Csr)  // the step's pattern: acc every third order
            return launch_iter_lazy(*c, s, (i & 1) ? V1 : V0, (i & 1) ? V0 : V1, acc, i % 3 == 2 ? 3 : 0,
                                    weight(c, 1), weight(c, 1), weight(c, 1));
        return launch_iter(*c, s, (i & 1) ? V1 : V0, (i & 1) ? V0 : V1, acc, weight(c, 1));
    };
    if (e == hipSuccess) e = one(0);  // untimed: pages in code and caches
    if (e == hipSuccess) e = hipEventRecord(c->ev_a, s);
    for (int i = 0; i < launches && e == hipSuccess; ++i) e = one(i + 1);
    if (e == hipSuccess) e = hipEventRecord(c->ev_b, s);
    if (e == hipSuccess) e = hipEventSynchronize(c->ev_b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->ev_a, c->ev_b);
    release(scratch);
    if (e != hipSuccess) return hip_fail(c, e, "chebtd_time_recursion_kernel");
    *ms_per_launch = (double)ms / launches;
    return CHEBTD_OK;
}

}  // extern "C"
