// Host side of the adjoint: storage schedules and the reverse sweep over
// time steps.  The forward run keeps psi at the start of every step; the
// backward run rebuilds that step's Chebyshev vectors from it (all M+1 of
// them, or in segments of about sqrt(M) orders from (v_{j-1}, v_j) pairs)
// and runs the reverse recursion, several levels per pass where it can
// (adjoint.hip).  The third schedule also keeps the step's last two vectors
// and regenerates the others downwards inside the reverse passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <string>
#include <vector>

#include "internal.h"
#include "pair.h"

namespace chebtd {
int fail(Ctx *c, int code, const std::string &msg);
int hip_fail(Ctx *c, hipError_t e, const char *what);
int ensure(Ctx *c, DevBuf &b, size_t bytes, const char *what);
void release(DevBuf &b);

struct AdjState {
    int64_t max_steps = 0;
    int mode = CHEBTD_ADJ_STEP;
    int seg = 1;          // orders per segment (sqrt mode)
    int M = 0;            // order the buffers were sized for
    int64_t plan_version = -1;
    int64_t last_K = 0;   // steps stored by the last checkpointing run
    int64_t ckpt_version = -1;
    int64_t ckpt_run = 0;  // number of that run (Ctx::run_seq), 0: none
    DevBuf ckpt;   // psi_s, s < max_steps
    DevBuf vbuf;   // recompute buffer
    DevBuf pairs;  // (v_{j-1}, v_j) per segment (sqrt mode)
    DevBuf u;      // two adjoint vectors
    DevBuf ends;   // (v_{M-1}, v_M) per step (reverse mode)
    // downward sweeps (reverse mode, and the sqrt mode where the deep walk
    // fits): levels per pass from level M-1 down, and in the sqrt mode the
    // pair slot each pass restarts from (-1: it continues from the pairs the
    // pass above regenerated)
    bool down = false;
    std::vector<int> rdepths, cpslot;
    DevBuf hpart;  // norm partials of the recomputation's head pass (unused)
};

void adj_destroy(Ctx *c)
{
    if (!c->adj) return;
    release(c->adj->ckpt);
    release(c->adj->vbuf);
    release(c->adj->pairs);
    release(c->adj->u);
    release(c->adj->ends);
    release(c->adj->hpart);
    delete c->adj;
    c->adj = nullptr;
}

// Start a checkpointing run of K steps: false if the storage is missing, too
// small or sized for another plan.  The run gets the next number; the
// adjoint refuses to run for any other.
bool adj_begin_run(Ctx *c, int64_t K)
{
    AdjState *a = c->adj;
    if (!a || K > a->max_steps || a->plan_version != c->plan_version) return false;
    a->last_K = K;
    a->ckpt_version = c->plan_version;
    a->ckpt_run = ++c->run_seq;
    return true;
}

// Checkpoint slot of `step` for a run of K steps, or null if the storage is
// missing or too small.
double2 *adj_checkpoint(Ctx *c, int64_t step, int64_t K)
{
    AdjState *a = c->adj;
    if (!a || K > a->max_steps || a->plan_version != c->plan_version) return nullptr;
    return static_cast<double2 *>(a->ckpt.p) + (size_t)step * (size_t)c->n;
}

// Number of the checkpointing run the adjoint would use now, 0 if none (no
// run since the storage was reserved, or the plan changed since).
int64_t adj_current_run(const Ctx *c)
{
    const AdjState *a = c->adj;
    if (!a || !c->has_plan || a->plan_version != c->plan_version || a->ckpt_version != c->plan_version ||
        a->ckpt_run == 0)
        return 0;
    return a->ckpt_run;
}

// Slot of (v_{M-1}, v_M) of `step` (2 n values) for the reverse schedule, or
// null when the adjoint storage does not keep them.
double2 *adj_step_ends(Ctx *c, int64_t step)
{
    AdjState *a = c->adj;
    if (!a || a->mode != CHEBTD_ADJ_REVERSE || a->plan_version != c->plan_version || step >= a->max_steps ||
        !a->ends.p)
        return nullptr;
    return static_cast<double2 *>(a->ends.p) + (size_t)step * 2 * (size_t)c->n;
}

}  // namespace chebtd

using namespace chebtd;
struct chebtd_ctx : public Ctx {};

namespace {

double2 conj_weight(const Ctx *c, int k)
{
    return make_double2(c->gamma[2 * (size_t)k], -c->gamma[2 * (size_t)k + 1]);
}

// The adjoint vectors in flight: u_{k+1} (uk1) and u_{k+2} (uk2, absent
// right after u_M), rotated through four buffers so that a two-level pass
// writes to buffers its neighbours are not reading.
struct URot {
    double2 *buf[4];
    double2 *uk1 = nullptr, *uk2 = nullptr;
    bool has2 = false;
    void start(double2 *uM)
    {
        uk1 = uM;
        uk2 = nullptr;
        has2 = false;
    }
    // two buffers holding neither uk1 nor uk2
    void spare(double2 **a, double2 **b) const
    {
        int got = 0;
        for (double2 *p : buf)
            if (p != uk1 && p != uk2) {
                (got == 0 ? *a : *b) = p;
                if (++got == 2) return;
            }
    }
};

// Orders per recomputation pass (each order stored): 6 on ribbons where the
// deep kernel's offsets fit, else 2 (a chain, one row, gains nothing from
// deeper passes: measured on MI355X); CHEBTD_REC_DEPTH overrides.
int rec_depth(const Ctx &c)
{
    int D = c.kind == HKind::Honeycomb ? 6 : 2;
    if (const char *env = std::getenv("CHEBTD_REC_DEPTH")) D = std::max(2, std::min(kMaxDepth, std::atoi(env)));
    if (!pair_supported(c)) return 1;
    const OpPair op = make_pair_op(c, 1);
    return deep_offsets_fit(op.W, op.L) ? D : 2;
}

// Adjoint levels per pass: 5 on ribbons, 2 on chains (measured on MI355X for
// the 256 x 4096 ribbon and the 65536-site chain: 5 levels per pass cut the
// ribbon's backward sweep from 151 to 94 ms, a chain only gets slower),
// limited by the lattice's offsets; CHEBTD_ADJ_DEPTH (2 .. 6) overrides.
int adj_depth(const Ctx &c)
{
    int D = c.kind == HKind::Honeycomb ? 5 : 2;
    if (const char *env = std::getenv("CHEBTD_ADJ_DEPTH")) D = std::max(2, std::min(kMaxDepth, std::atoi(env)));
    if (!pair_supported(c)) return 1;
    while (D > 2 && !adj_deep_fits(c, D)) --D;
    return D;
}

// Reverse sweep of one step for levels k = kend-1 .. kbeg, with the forward
// vectors v_k available as vk(k).  Levels k .. k-D+1 >= 1 go D per pass on
// chains and ribbons where their forward vectors are stored n apart, else
// two per pass (pair_supported); a level left alone writes u_k over u_{k+2}
// (own site only); level 0 writes u_0 over gbar.
template <class VK>
hipError_t sweep_levels(Ctx *c, hipStream_t s, int kbeg, int kend, VK vk, double2 *gbar, double *grad, URot &u)
{
    const bool pairs = pair_supported(*c);
    const int D = adj_depth(*c);
    const int64_t n = c->n;
    auto spaced = [&](int lo, int hi) {  // v_lo .. v_hi stored n apart
        for (int k = lo + 1; k <= hi; ++k)
            if (vk(k) != vk(lo) + (k - lo) * n) return false;
        return true;
    };
    hipError_t e = hipSuccess;
    int k = kend - 1;
    while (k >= kbeg && e == hipSuccess) {
        if (D > 2 && k - D + 1 >= std::max(kbeg, 1) && spaced(k - D + 1, k)) {
            double2 *o1, *o2;
            u.spare(&o1, &o2);
            double2 cw[kMaxDepth];
            for (int j = 1; j <= D; ++j) cw[j - 1] = conj_weight(c, k - j + 1);
            e = launch_adj_deep(*c, s, D, c->deep_rows[D], u.has2 ? u.uk2 : nullptr, u.uk1, o1, o2, gbar, grad,
                                vk(k - D + 1), cw);
            u.uk2 = o1;  // u_{k-D+2}
            u.uk1 = o2;  // u_{k-D+1}
            u.has2 = true;
            k -= D;
        } else if (pairs && k - 1 >= std::max(kbeg, 1)) {
            double2 *o1, *o2;
            u.spare(&o1, &o2);
            e = launch_adj_pair(*c, s, u.has2, u.uk2, u.uk1, o1, o2, gbar, vk(k), vk(k - 1), conj_weight(c, k),
                                conj_weight(c, k - 1), grad);
            u.uk2 = o1;  // u_k
            u.uk1 = o2;  // u_{k-1}
            u.has2 = true;
            k -= 2;
        } else if (k >= 1) {
            double2 *out = u.uk2;
            if (!u.has2) {
                double2 *o2;
                u.spare(&out, &o2);
            }
            e = launch_adj_level(*c, s, u.uk1, u.uk2, gbar, out, vk(k), conj_weight(c, k), 2.0, u.has2, grad);
            u.uk2 = u.uk1;
            u.uk1 = out;
            u.has2 = true;
            k -= 1;
        } else {
            e = launch_adj_level(*c, s, u.uk1, u.uk2, gbar, gbar, vk(0), conj_weight(c, 0), 1.0, u.has2, grad);
            k -= 1;
        }
    }
    return e;
}

// Levels per pass of the reverse schedule (2 .. kMaxRevDepth, 5 being the
// most that keeps both recursions in registers without spilling): 5 on
// ribbons, 3 on chains (measured on MI355X, 256 x 4096 ribbon and 65536-site
// chain at order 64: 0.50 and 0.23 ms per step; 4 levels 0.56 and 0.30,
// chains at 5 levels 0.29); CHEBTD_REV_DEPTH overrides.
int rev_depth(const Ctx &c)
{
    int D = c.kind == HKind::Honeycomb ? 5 : 3;
    if (const char *env = std::getenv("CHEBTD_REV_DEPTH")) D = std::atoi(env);
    return std::max(2, std::min(kMaxRevDepth, D));
}

// Rows per wavefront chunk of a reverse pass of depth D, with rows + 2 (D - 1)
// a multiple of the 6-iteration body.  Up to 4M sites the chunk count decides:
// at 1M sites 22-row chunks give 5-level passes about one wavefront per SIMD
// (two fit at 236 VGPRs) and ran 0.50 ms per step against 0.52 for 10 rows and
// 0.61 for 16 (unevenly 1 or 2 per SIMD); past it the propagation's deep-pass
// heights.  CHEBTD_REV_ROWS overrides.
int rev_rows(const Ctx &c, int D)
{
    if (const char *env = std::getenv("CHEBTD_REV_ROWS")) return std::max(1, std::atoi(env));
    static const int small[kMaxRevDepth + 1] = {0, 0, 10, 14, 24, 22};
    if (c.n >= (int64_t(1) << 22) && D >= 3 && c.deep_rows[D] > 0) return c.deep_rows[D];
    return small[D];
}

// Levels per pass of a downward sweep from level M-1 to level 0: rev_depth
// each, and no pass of a single level (the walk needs two).
std::vector<int> rev_pass_depths(const Ctx &c)
{
    std::vector<int> depths;
    const int Dm = rev_depth(c);
    for (int rem = c.M; rem > 0;) {
        int d = std::min(Dm, rem);
        if (rem - d == 1) d = rem <= kMaxRevDepth ? rem : d - 1;
        depths.push_back(d);
        rem -= d;
    }
    return depths;
}

// The sqrt mode's forward pass of one step on the downward path: from psi_s,
// the passes of the downward sweep in reverse order (so every pass ends on
// an order where a downward pass starts), each advancing its orders without
// the accumulator (the deep walk with no acc buffer reads and writes none of
// it: 72 B per site and pass).  A pass whose end starts a restarting
// downward pass writes its (v_{e-1}, v_e) into that pair slot; the others
// rotate through four scratch vectors.  The last pass ends on (v_{M-1}, v_M)
// in slot 0.
hipError_t recompute_pairs(Ctx *c, hipStream_t s, const double2 *psi_s, double2 *const vr[4])
{
    AdjState *a = c->adj;
    const int64_t n = c->n;
    const int P = (int)a->rdepths.size();
    double2 *pairs = static_cast<double2 *>(a->pairs.p);
    const double2 *gam = reinterpret_cast<const double2 *>(c->gamma.data());
    const double2 *in1 = nullptr, *in2 = psi_s;  // (v_{k-1}, v_k)
    int k = 0;
    hipError_t e = hipSuccess;
    for (int f = 0; f < P && e == hipSuccess; ++f) {
        const int p = P - 1 - f, d = a->rdepths[p];
        double2 *o1 = nullptr, *o2 = nullptr;
        if (a->cpslot[p] >= 0) {
            o1 = pairs + (size_t)(2 * a->cpslot[p]) * n;
            o2 = o1 + n;
        } else {
            for (int j = 0; j < 4; ++j) {
                if (vr[j] == in1 || vr[j] == in2) continue;
                if (!o1)
                    o1 = vr[j];
                else if (!o2)
                    o2 = vr[j];
            }
        }
        if (d == 2)
            e = launch_recompute_pair(*c, s, k == 0, in1, in2, o1, o2);
        else
            e = launch_deep(*c, s, d, c->deep_rows[d], k == 0, in1, in2, o1, o2, nullptr, gam + k, nullptr,
                            static_cast<double *>(a->hpart.p), nullptr);
        in1 = o1;
        in2 = o2;
        k += d;
    }
    if (e == hipSuccess && k != c->M) e = hipErrorInvalidValue;
    return e;
}

// The downward schedules over all steps.  Per step, from (v_{M-1}, v_M) --
// stored by the forward run (reverse mode) or rebuilt from psi_s by
// recompute_pairs (sqrt mode) -- passes of levels k .. k-d+1 regenerate the
// forward vectors downwards beside the adjoint recursion; in the sqrt mode
// every pass with a pair slot starts from the stored pair instead of the
// regenerated one (the pass above then stores no forward vectors).  The pass
// holding level 0 writes u_0, the next step's gbar, into the other of two
// gbar buffers (the pass still reads the current one around its rows).
// M = 1 has level 0 alone.
hipError_t reverse_sweep(Ctx *c, hipStream_t s, double2 *gbar_user, double *grad, URot &u)
{
    AdjState *a = c->adj;
    const bool seg = a->mode == CHEBTD_ADJ_SQRTM;
    const int M = c->M;
    const int64_t n = c->n;
    double2 *vb = static_cast<double2 *>(a->vbuf.p);
    double2 *const vr[4] = {vb, vb + n, vb + 2 * n, vb + 3 * n};
    double2 *pairs = static_cast<double2 *>(a->pairs.p);
    double2 *gcur = gbar_user, *gnext = vb + 4 * n;
    const std::vector<int> &depths = a->rdepths;
    const int P = (int)depths.size();
    hipError_t e = hipSuccess;
    for (int64_t st = a->last_K - 1; st >= 0 && e == hipSuccess; --st) {
        double2 *psi_s = static_cast<double2 *>(a->ckpt.p) + (size_t)st * n;
        u.start(u.buf[0]);
        e = launch_adj_init(s, gcur, conj_weight(c, M), u.uk1, n);  // u_M
        if (e != hipSuccess) break;
        if (M == 1) {
            e = sweep_levels(c, s, 0, 1, [&](int) { return psi_s; }, gcur, grad, u);
            continue;
        }
        const double2 *v1, *v0;  // v_{k+1}, v_k for k = M-1
        if (seg) {
            e = recompute_pairs(c, s, psi_s, vr);
            if (e != hipSuccess) break;
            v1 = pairs + n;
            v0 = pairs;
        } else {
            double2 *ends = adj_step_ends(c, st);
            if (!ends) return hipErrorInvalidValue;
            v1 = ends + n;
            v0 = ends;
        }
        int k = M - 1;
        for (int i = 0; i < P; ++i) {
            const int d = depths[i];
            if (seg && a->cpslot[i] >= 0) {
                const double2 *slot = pairs + (size_t)(2 * a->cpslot[i]) * n;
                v1 = slot + n;
                v0 = slot;
            }
            RevPass p{};
            p.last0 = k - d + 1 == 0;
            double2 *o1, *o2;
            u.spare(&o1, &o2);
            p.uk2 = u.has2 ? u.uk2 : nullptr;
            p.uk1 = u.uk1;
            p.out1 = p.last0 ? nullptr : o1;
            p.out2 = p.last0 ? gnext : o2;
            p.gbar = gcur;
            p.grad = grad;
            p.v1 = v1;
            p.v0 = v0;
            const bool restart_next = seg && i + 1 < P && a->cpslot[i + 1] >= 0;
            if (!p.last0 && !restart_next) {
                for (double2 *w : vr) {
                    if (w == v1 || w == v0) continue;
                    if (!p.vout1)
                        p.vout1 = w;
                    else if (!p.vout2)
                        p.vout2 = w;
                }
            }
            for (int j = 1; j <= d; ++j) p.cw[j - 1] = conj_weight(c, k - j + 1);
            e = launch_rev_deep(*c, s, d, rev_rows(*c, d), p);
            if (e != hipSuccess) break;
            u.uk2 = o1;  // u_{k-d+2}
            u.uk1 = o2;  // u_{k-d+1}
            u.has2 = true;
            v1 = p.vout1;  // v_{k-d+1}
            v0 = p.vout2;  // v_{k-d}
            k -= d;
        }
        if (e == hipSuccess && k != -1) e = hipErrorInvalidValue;
        std::swap(gcur, gnext);
    }
    if (e == hipSuccess && gcur != gbar_user) e = launch_copy(s, gcur, gbar_user, n);
    return e;
}

}  // namespace

extern "C" {

int chebtd_reserve_adjoint(chebtd_ctx *ctx, int64_t max_steps, int mode)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = static_cast<Ctx *>(ctx);
    if (!c->has_plan || (c->kind != HKind::Chain && c->kind != HKind::Honeycomb))
        return fail(c, CHEBTD_E_STATE, "chebtd_reserve_adjoint: needs a plan for a chain or honeycomb H");
    if (max_steps < 1 || (mode != CHEBTD_ADJ_STEP && mode != CHEBTD_ADJ_SQRTM && mode != CHEBTD_ADJ_REVERSE))
        return fail(c, CHEBTD_E_ARG, "chebtd_reserve_adjoint: need max_steps >= 1 and a known mode");
    if (mode == CHEBTD_ADJ_REVERSE && !rev_deep_fits(*c))
        return fail(c, CHEBTD_E_ARG,
                    "chebtd_reserve_adjoint: CHEBTD_ADJ_REVERSE needs (W + 14) L 16 B <= 2^31 (the deep walk's offsets)");
    if (!c->adj) c->adj = new (std::nothrow) AdjState();
    if (!c->adj) return fail(c, CHEBTD_E_OOM, "adjoint state");
    AdjState *a = c->adj;
    const size_t vb = (size_t)c->n * sizeof(double2);
    const int M = c->M;
    a->mode = mode;
    a->max_steps = max_steps;
    a->M = M;
    // ceil(sqrt(M)) orders per segment, rounded up to even so that the
    // two-orders-per-pass recomputation ends exactly on segment boundaries
    a->seg = std::max(1, (int)std::ceil(std::sqrt((double)std::max(M, 1))));
    if (pair_supported(*c)) a->seg += a->seg & 1;
    // the reverse mode, and the sqrt mode where the deep walk fits, sweep
    // downwards (M >= 2; M = 1 is level 0 alone)
    a->down = mode == CHEBTD_ADJ_REVERSE || (mode == CHEBTD_ADJ_SQRTM && rev_deep_fits(*c) && M >= 2);
    a->rdepths = a->down ? rev_pass_depths(*c) : std::vector<int>();
    a->cpslot.assign(a->rdepths.size(), -1);
    int rc;
    if ((rc = ensure(c, a->ckpt, vb * (size_t)max_steps, "adjoint checkpoints"))) return rc;
    if ((rc = ensure(c, a->u, 4 * vb, "adjoint vectors"))) return rc;
    if (mode == CHEBTD_ADJ_STEP) {
        release(a->pairs);
        release(a->ends);
        if ((rc = ensure(c, a->vbuf, vb * (size_t)(M + 1), "recompute buffer"))) return rc;
    } else if (mode == CHEBTD_ADJ_REVERSE) {
        // four vectors for the downward pairs, one for the other gbar
        release(a->pairs);
        if ((rc = ensure(c, a->ends, 2 * vb * (size_t)max_steps, "step-end pairs"))) return rc;
        if ((rc = ensure(c, a->vbuf, 5 * vb, "downward vectors"))) return rc;
    } else if (a->down) {
        // a pair slot for the top pass and then one each time at least
        // ceil(sqrt(M)) levels have passed since the last slot; four vectors
        // for the forward pass's and the downward pairs, one for the other gbar
        release(a->ends);
        const int S = std::max(1, (int)std::ceil(std::sqrt((double)M)));
        int nslot = 0, since = 0;
        for (size_t i = 0; i < a->rdepths.size(); ++i) {
            if (i == 0 || since >= S) {
                a->cpslot[i] = nslot++;
                since = 0;
            }
            since += a->rdepths[i];
        }
        if ((rc = ensure(c, a->pairs, vb * 2 * (size_t)std::max(nslot, 1), "checkpoint pairs"))) return rc;
        if ((rc = ensure(c, a->vbuf, 5 * vb, "downward vectors"))) return rc;
        const int dh = a->rdepths.empty() ? 2 : a->rdepths.back();  // the forward pass's head
        const int64_t hb = dh >= 3 ? deep_grid_blocks(*c, c->deep_rows[dh], dh) : 1;
        if ((rc = ensure(c, a->hpart, (size_t)std::max<int64_t>(hb, 1) * 2 * sizeof(double), "head partials")))
            return rc;
    } else {
        release(a->ends);
        const int nseg = (M + a->seg - 1) / a->seg;
        if ((rc = ensure(c, a->pairs, vb * 2 * (size_t)std::max(nseg, 1), "segment pairs"))) return rc;
        if ((rc = ensure(c, a->vbuf, vb * (size_t)(a->seg + 1), "segment buffer"))) return rc;
    }
    a->plan_version = c->plan_version;
    a->last_K = 0;
    a->ckpt_version = -1;
    a->ckpt_run = 0;
    return CHEBTD_OK;
}

int chebtd_checkpoint_run(const chebtd_ctx *ctx, int64_t *run_id)
{
    if (!ctx || !run_id) return fail(nullptr, CHEBTD_E_ARG, "chebtd_checkpoint_run: null pointer");
    *run_id = adj_current_run(static_cast<const Ctx *>(ctx));
    return CHEBTD_OK;
}

int chebtd_adjoint(chebtd_ctx *ctx, double *gbar_dev, double *dLdV_dev)
{
    return chebtd_adjoint_run(ctx, 0, gbar_dev, dLdV_dev);
}

int chebtd_adjoint_run(chebtd_ctx *ctx, int64_t run_id, double *gbar_dev, double *dLdV_dev)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = static_cast<Ctx *>(ctx);
    AdjState *a = c->adj;
    if (!gbar_dev || !dLdV_dev) return fail(c, CHEBTD_E_ARG, "chebtd_adjoint: null pointer");
    const int64_t cur = adj_current_run(c);
    if (cur == 0)
        return fail(c, CHEBTD_E_STATE,
                    "chebtd_adjoint: run chebtd_propagate with CHEBTD_KEEP_CHECKPOINTS on the current plan first");
    if (run_id != 0 && run_id != cur)
        return fail(c, CHEBTD_E_STATE,
                    "chebtd_adjoint: the checkpoints of run " + std::to_string(run_id) +
                        " were overwritten (the stored run is " + std::to_string(cur) + ")");
    // a run of zero steps: psi_K = psi_0, so gbar passes through and dL/dV
    // gains nothing
    if (a->last_K == 0) return CHEBTD_OK;
    hipStream_t s = c->stream;
    const int M = c->M;
    const int64_t n = c->n;
    double2 *gbar = reinterpret_cast<double2 *>(gbar_dev);
    double2 *ck = static_cast<double2 *>(a->ckpt.p);
    double2 *vb = static_cast<double2 *>(a->vbuf.p);
    URot urot;
    for (int q = 0; q < 4; ++q) urot.buf[q] = static_cast<double2 *>(a->u.p) + (size_t)q * n;
    const bool pairs_on = pair_supported(*c);
    hipError_t e = hipSuccess;
    if (a->down && M >= 1) {
        e = reverse_sweep(c, s, gbar, dLdV_dev, urot);
        if (e != hipSuccess) return hip_fail(c, e, "chebtd_adjoint (downward schedule)");
        return CHEBTD_OK;
    }
    for (int64_t st = a->last_K - 1; st >= 0 && e == hipSuccess; --st) {
        double2 *psi_s = ck + (size_t)st * n;
        if (M == 0) {
            e = launch_scale_copy(s, gbar, gbar, conj_weight(c, 0), n);
            continue;
        }
        // u_M = conj(gamma_M) gbar
        urot.start(urot.buf[0]);
        e = launch_adj_init(s, gbar, conj_weight(c, M), urot.uk1, n);
        if (e != hipSuccess) break;
        if (a->mode == CHEBTD_ADJ_STEP) {
            // v_0 = psi_s (the checkpoint itself), v_1 .. v_M into the buffer
            auto vk = [&](int k) -> double2 * { return k == 0 ? psi_s : vb + (size_t)k * n; };
            int k = 0;  // v_0 .. v_k are known
            const int DR = rec_depth(*c);
            if (DR > 2 && M - 1 >= DR) {
                // D orders per pass, every one stored
                double2 *all[kMaxDepth];
                for (int j = 0; j < DR; ++j) all[j] = vk(j + 1);
                e = launch_recompute_deep(*c, s, DR, c->deep_rows[DR], true, nullptr, psi_s, all);
                k = DR;
                for (; k + DR <= M - 1 && e == hipSuccess; k += DR) {
                    for (int j = 0; j < DR; ++j) all[j] = vk(k + j + 1);
                    e = launch_recompute_deep(*c, s, DR, c->deep_rows[DR], false, vk(k - 1), vk(k), all);
                }
                for (; k + 2 <= M - 1 && e == hipSuccess; k += 2)
                    e = launch_recompute_pair(*c, s, false, vk(k - 1), vk(k), vk(k + 1), vk(k + 2));
            } else if (pairs_on && M - 1 >= 2) {
                e = launch_recompute_pair(*c, s, true, nullptr, psi_s, vk(1), vk(2));
                k = 2;
                for (; k + 2 <= M - 1 && e == hipSuccess; k += 2)
                    e = launch_recompute_pair(*c, s, false, vk(k - 1), vk(k), vk(k + 1), vk(k + 2));
            }
            for (; k + 1 <= M - 1 && e == hipSuccess; ++k)
                e = launch_recompute(*c, s, vk(k), k ? vk(k - 1) : nullptr, vk(k + 1), k == 0);
            if (e == hipSuccess) e = sweep_levels(c, s, 0, M, vk, gbar, dLdV_dev, urot);
        } else {
            // forward pass keeping (v_{qS-1}, v_{qS}) for segments q >= 1
            const int S = a->seg, nseg = (M + S - 1) / S;
            double2 *pairs = static_cast<double2 *>(a->pairs.p);
            const int kmax = (nseg - 1) * S;  // the last boundary order needed
            if (pairs_on && S % 2 == 0 && S >= 4) {
                // two orders per pass; a pass that ends on a boundary writes
                // straight into that boundary's pair, the others rotate
                // through four scratch vectors
                const double2 *in1 = nullptr, *in2 = psi_s;  // (v_{k-1}, v_k)
                for (int k = 0; k < kmax && e == hipSuccess; k += 2) {
                    double2 *o1 = nullptr, *o2 = nullptr;
                    if ((k + 2) % S == 0) {
                        const int q = (k + 2) / S;
                        o1 = pairs + (size_t)(2 * q) * n;
                        o2 = pairs + (size_t)(2 * q + 1) * n;
                    } else {
                        for (int j = 0; j < 4; ++j) {
                            double2 *p = vb + (size_t)j * n;
                            if (p == in1 || p == in2) continue;
                            if (!o1)
                                o1 = p;
                            else if (!o2)
                                o2 = p;
                        }
                    }
                    e = launch_recompute_pair(*c, s, k == 0, in1, in2, o1, o2);
                    in1 = o1;
                    in2 = o2;
                }
                // segments in reverse: v_{k0-1}, v_{k0} come from the pair
                // storage, v_{k0+1} .. v_{k1-1} into buffer slots 1 ..
                for (int q = nseg - 1; q >= 0 && e == hipSuccess; --q) {
                    const int k0 = q * S, k1 = std::min(k0 + S, M);
                    double2 *prev = q > 0 ? pairs + (size_t)(2 * q) * n : nullptr;
                    double2 *first = q > 0 ? pairs + (size_t)(2 * q + 1) * n : psi_s;
                    auto vk = [&](int k) -> double2 * { return k == k0 ? first : vb + (size_t)(k - k0) * n; };
                    auto vkm = [&](int k) -> double2 * { return k == k0 ? prev : vk(k - 1); };
                    int j = 0;  // v_{k0} .. v_{k0+j} are known
                    for (; k0 + j + 2 <= k1 - 1 && e == hipSuccess; j += 2)
                        e = launch_recompute_pair(*c, s, k0 + j == 0, vkm(k0 + j), vk(k0 + j), vk(k0 + j + 1),
                                                  vk(k0 + j + 2));
                    if (k0 + j + 1 <= k1 - 1 && e == hipSuccess)
                        e = launch_recompute(*c, s, vk(k0 + j), vkm(k0 + j), vk(k0 + j + 1), k0 + j == 0);
                    if (e == hipSuccess) e = sweep_levels(c, s, k0, k1, vk, gbar, dLdV_dev, urot);
                }
                continue;
            }
            double2 *w0 = vb, *w1 = vb + n, *w2 = vb + 2 * (size_t)n;  // rotating scratch
            // v_0 = psi_s; compute up to v_{(nseg-1) S}
            const double2 *km1 = nullptr, *kc = psi_s;
            double2 *rot[3] = {w0, w1, w2};
            for (int k = 0; k < kmax && e == hipSuccess; ++k) {
                double2 *dst = rot[k % 3];
                e = launch_recompute(*c, s, kc, km1, dst, k == 0);
                km1 = kc;
                kc = dst;
                const int kk = k + 1;  // order just formed
                if (kk % S == 0 && e == hipSuccess) {
                    const int q = kk / S;
                    e = hipMemcpyAsync(pairs + (size_t)(2 * q) * n, km1, n * sizeof(double2),
                                       hipMemcpyDeviceToDevice, s);
                    if (e == hipSuccess)
                        e = hipMemcpyAsync(pairs + (size_t)(2 * q + 1) * n, kc, n * sizeof(double2),
                                           hipMemcpyDeviceToDevice, s);
                }
            }
            // segments in reverse: rebuild v_{qS} .. v_{min(qS+S, M)-1}
            for (int q = nseg - 1; q >= 0 && e == hipSuccess; --q) {
                const int k0 = q * S, k1 = std::min(k0 + S, M);
                // buffer slot j holds v_{k0 + j}; slot S holds v_{k0-1}
                auto vk = [&](int k) -> double2 * {
                    if (k == 0) return psi_s;
                    return vb + (size_t)(k - k0) * n;
                };
                double2 *prev = nullptr;
                if (q > 0) {
                    e = hipMemcpyAsync(vb + (size_t)S * n, pairs + (size_t)(2 * q) * n, n * sizeof(double2),
                                       hipMemcpyDeviceToDevice, s);
                    if (e == hipSuccess)
                        e = hipMemcpyAsync(vb, pairs + (size_t)(2 * q + 1) * n, n * sizeof(double2),
                                           hipMemcpyDeviceToDevice, s);
                    prev = vb + (size_t)S * n;
                }
                for (int k = k0; k + 1 <= k1 - 1 && e == hipSuccess; ++k) {
                    const double2 *cur = vk(k);
                    const double2 *km = (k == k0) ? prev : vk(k - 1);
                    e = launch_recompute(*c, s, cur, km, vb + (size_t)(k + 1 - k0) * n, k == 0);
                }
                if (e == hipSuccess) e = sweep_levels(c, s, k0, k1, vk, gbar, dLdV_dev, urot);
            }
        }
    }
    if (e != hipSuccess) return hip_fail(c, e, "chebtd_adjoint");
    return CHEBTD_OK;
}

}  // extern "C"
