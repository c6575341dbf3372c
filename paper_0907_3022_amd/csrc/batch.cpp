// Host side of the batched ribbon path: per-system plans, schedule tables,
// hipGraph capture of step pairs, and the autotuner that times candidate
// schedules on the real batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "batch_internal.h"
#include "internal.h"
#include "pair.h"

namespace chebtd {
int fail(Ctx *c, int code, const std::string &msg);
int hip_fail(Ctx *c, hipError_t e, const char *what);
int ensure(Ctx *c, DevBuf &b, size_t bytes, const char *what);
void release(DevBuf &b);

struct BatchState {
    int nsys = 0;
    double dt = 0.0;
    std::vector<SysDev> sys;       // indexed by system id
    std::vector<int> M;            // order per system
    std::vector<int64_t> nsites;   // sites per system
    std::vector<int32_t> order;    // system ids by M descending
    std::vector<double> gamma;     // concatenated weights (interleaved)
    DevBuf sys_dev, gamma_dev, work;
    // schedule
    int mode = CHEBTD_SCHED_LEVELS, tile = 2048, block = 256, wg_per_cu = 2;
    int nlevels = 1;
    std::vector<int64_t> level_blocks;  // blocks launched at each level
    DevBuf blk_sys, blk_tile, q_level_off, q_level_active, q_tile_prefix, q_order;
    QueueDev q{};
    int64_t nblocks = 0;
    // pairs schedule: blocks per pair level (active systems are a prefix of
    // `order`), and the tail tiles of systems with odd M
    bool pairs_ok = false;
    std::vector<int64_t> pair_level_blocks;
    DevBuf pblk_sys, pblk_wave0, tblk_sys, tblk_tile;
    int64_t ntail_blocks = 0;
    // deep schedule: each system takes the fewest passes of deep_D or
    // deep_D + 1 orders that cover its M (deep_D + 1 first), then two-order
    // passes while it has two or more orders left, then the tail if one is
    // left; one launch per (pass, depth) over the systems it concerns, and
    // one per two-order pass (explicit block lists, concatenated)
    bool deep_ok = false;
    int deep_D = 5;
    struct DeepLaunch {
        int pass, depth;
        int64_t off, count;
    };
    std::vector<DeepLaunch> deep_launches;
    std::vector<int64_t> deep_pair_off;
    DevBuf dblk_sys, dblk_wave0, dpblk_sys, dpblk_wave0, dtblk_sys, dtblk_tile;
    int64_t ndtail_blocks = 0;
    DevBuf head, done, flag;
    int64_t spin_limit = 0;  // wall-clock ticks a dependency wait may take
    hipGraphExec_t graph = nullptr;
    hipStream_t cap = nullptr;
    // re-binding the systems' states: a pinned mirror of the system table,
    // and an event on the last upload from it
    SysDev *sys_pinned = nullptr;
    hipEvent_t sys_ev = nullptr;
    bool sys_ev_pending = false;
};

static void drop_graph(BatchState *b)
{
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
}

void batch_destroy(Ctx *c)
{
    BatchState *b = c->batch;
    if (!b) return;
    drop_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->sys_ev) {
        (void)hipEventSynchronize(b->sys_ev);
        (void)hipEventDestroy(b->sys_ev);
    }
    if (b->sys_pinned) (void)hipHostFree(b->sys_pinned);
    for (DevBuf *d : {&b->sys_dev, &b->gamma_dev, &b->work, &b->blk_sys, &b->blk_tile, &b->q_level_off,
                      &b->q_level_active, &b->q_tile_prefix, &b->q_order, &b->pblk_sys, &b->pblk_wave0,
                      &b->tblk_sys, &b->tblk_tile, &b->dblk_sys, &b->dblk_wave0, &b->dpblk_sys, &b->dpblk_wave0,
                      &b->dtblk_sys, &b->dtblk_tile, &b->head, &b->done, &b->flag})
        release(*d);
    delete b;
    c->batch = nullptr;
}

static int upload(Ctx *c, DevBuf &d, const void *src, size_t bytes, const char *what)
{
    int rc = ensure(c, d, std::max<size_t>(bytes, 8), what);
    if (rc) return rc;
    hipError_t e = hipMemcpy(d.p, src, bytes, hipMemcpyHostToDevice);
    return e == hipSuccess ? CHEBTD_OK : hip_fail(c, e, what);
}

// Rebuild the tile tables for the current tile size.
static int build_tables(Ctx *c, BatchState *b)
{
    const int ns = b->nsys;
    std::vector<int64_t> tiles(ns);
    for (int s = 0; s < ns; ++s) {
        tiles[s] = (b->nsites[s] + b->tile - 1) / b->tile;
        if (tiles[s] > INT32_MAX) return fail(c, CHEBTD_E_ARG, "batch: too many tiles in one system");
        b->sys[s].ntiles = (int32_t)tiles[s];
    }
    int Mmax = 0;
    for (int s = 0; s < ns; ++s) Mmax = std::max(Mmax, b->M[s]);
    b->nlevels = std::max(1, Mmax);
    std::vector<int64_t> prefix(ns + 1, 0);
    for (int j = 0; j < ns; ++j) prefix[j + 1] = prefix[j] + tiles[b->order[j]];
    b->nblocks = prefix[ns];
    if (b->nblocks > INT32_MAX) return fail(c, CHEBTD_E_ARG, "batch: too many tiles");
    std::vector<int32_t> bsys((size_t)b->nblocks), btile((size_t)b->nblocks);
    for (int j = 0; j < ns; ++j)
        for (int64_t t = 0; t < tiles[b->order[j]]; ++t) {
            bsys[(size_t)(prefix[j] + t)] = b->order[j];
            btile[(size_t)(prefix[j] + t)] = (int32_t)t;
        }
    std::vector<int32_t> active(b->nlevels);
    std::vector<int64_t> loff(b->nlevels + 1, 0);
    b->level_blocks.assign(b->nlevels, 0);
    for (int k = 0; k < b->nlevels; ++k) {
        int cnt = 0;
        for (int j = 0; j < ns; ++j)
            if (k == 0 || b->M[b->order[j]] > k) ++cnt;
        active[k] = cnt;
        b->level_blocks[k] = prefix[cnt];
        loff[k + 1] = loff[k] + prefix[cnt];
    }
    // pairs schedule: level p runs the systems with M >= 2p + 2
    std::vector<int32_t> psys, pw0, tsys, ttile;
    b->pair_level_blocks.clear();
    if (b->pairs_ok) {
        std::vector<int64_t> pprefix(ns + 1, 0);
        for (int j = 0; j < ns; ++j) {
            const SysDev &sd = b->sys[b->order[j]];
            const int64_t waves = (int64_t)sd.nstrips * sd.nchunks;
            const int64_t nbk = (waves + 3) / 4;
            for (int64_t q = 0; q < nbk; ++q) {
                psys.push_back(b->order[j]);
                pw0.push_back((int32_t)(4 * q));
            }
            pprefix[j + 1] = pprefix[j] + nbk;
        }
        if (pprefix[ns] > INT32_MAX) return fail(c, CHEBTD_E_ARG, "batch: too many wavefronts");
        for (int p = 0; 2 * p + 2 <= Mmax; ++p) {
            int cnt = 0;
            for (int j = 0; j < ns; ++j)
                if (b->M[b->order[j]] >= 2 * p + 2) ++cnt;
            b->pair_level_blocks.push_back(pprefix[cnt]);
        }
        for (int s = 0; s < ns; ++s)
            if (b->M[s] & 1)
                for (int64_t t = 0; t < tiles[s]; ++t) {
                    tsys.push_back(s);
                    ttile.push_back((int32_t)t);
                }
    }
    b->ntail_blocks = (int64_t)tsys.size();
    // deep schedule tables
    std::vector<int32_t> dsys, dw0, dpsys, dpw0, dtsys, dttile;
    b->deep_launches.clear();
    b->deep_pair_off.assign(1, 0);
    if (b->deep_ok) {
        const int D = b->deep_D, E = D + 1;
        int maxpass = 0, maxrest = 0;
        for (int s = 0; s < ns; ++s) {
            maxpass = std::max(maxpass, b->sys[s].ndeep);
            maxrest = std::max(maxrest, b->M[s] - b->sys[s].kdeep);
        }
        for (int p = 0; p < maxpass; ++p)
            for (int depth : {E, D}) {
                const int64_t off = (int64_t)dsys.size();
                for (int j = 0; j < ns; ++j) {
                    const int sid = b->order[j];
                    const SysDev &sd = b->sys[sid];
                    if (p >= sd.ndeep || (p < sd.ndeep_ext ? E : D) != depth) continue;
                    const bool ext = depth != D;
                    const int64_t nbk = ((int64_t)(ext ? sd.dnstrips_ext : sd.dnstrips) *
                                             (ext ? sd.dnchunks_ext : sd.dnchunks) +
                                         3) /
                                        4;
                    for (int64_t w = 0; w < nbk; ++w) {
                        dsys.push_back(sid);
                        dw0.push_back((int32_t)(4 * w));
                    }
                }
                if ((int64_t)dsys.size() > off) b->deep_launches.push_back({p, depth, off, (int64_t)dsys.size() - off});
            }
        if ((int64_t)dsys.size() > INT32_MAX) return fail(c, CHEBTD_E_ARG, "batch: too many wavefronts");
        for (int q = 0; 2 * q + 2 <= maxrest; ++q) {
            for (int j = 0; j < ns; ++j) {
                const int sid = b->order[j];
                const SysDev &sd = b->sys[sid];
                if (b->M[sid] - sd.kdeep < 2 * q + 2) continue;
                const int64_t nbk = ((int64_t)sd.nstrips * sd.nchunks + 3) / 4;
                for (int64_t w = 0; w < nbk; ++w) {
                    dpsys.push_back(sid);
                    dpw0.push_back((int32_t)(4 * w));
                }
            }
            b->deep_pair_off.push_back((int64_t)dpsys.size());
        }
        if ((int64_t)dpsys.size() > INT32_MAX) return fail(c, CHEBTD_E_ARG, "batch: too many wavefronts");
        for (int s = 0; s < ns; ++s)
            if ((b->M[s] - b->sys[s].kdeep) & 1)
                for (int64_t t = 0; t < tiles[s]; ++t) {
                    dtsys.push_back(s);
                    dttile.push_back((int32_t)t);
                }
    }
    b->ndtail_blocks = (int64_t)dtsys.size();
    int rc;
    if (b->pairs_ok &&
        ((rc = upload(c, b->pblk_sys, psys.data(), psys.size() * 4, "pair block table")) ||
         (rc = upload(c, b->pblk_wave0, pw0.data(), pw0.size() * 4, "pair wavefront table")) ||
         (rc = upload(c, b->tblk_sys, tsys.data(), tsys.size() * 4, "tail block table")) ||
         (rc = upload(c, b->tblk_tile, ttile.data(), ttile.size() * 4, "tail tile table"))))
        return rc;
    if (b->deep_ok &&
        ((rc = upload(c, b->dblk_sys, dsys.data(), dsys.size() * 4, "deep block table")) ||
         (rc = upload(c, b->dblk_wave0, dw0.data(), dw0.size() * 4, "deep wavefront table")) ||
         (rc = upload(c, b->dpblk_sys, dpsys.data(), dpsys.size() * 4, "deep pair block table")) ||
         (rc = upload(c, b->dpblk_wave0, dpw0.data(), dpw0.size() * 4, "deep pair wavefront table")) ||
         (rc = upload(c, b->dtblk_sys, dtsys.data(), dtsys.size() * 4, "deep tail block table")) ||
         (rc = upload(c, b->dtblk_tile, dttile.data(), dttile.size() * 4, "deep tail tile table"))))
        return rc;
    if ((rc = upload(c, b->blk_sys, bsys.data(), bsys.size() * 4, "batch block table")) ||
        (rc = upload(c, b->blk_tile, btile.data(), btile.size() * 4, "batch tile table")) ||
        (rc = upload(c, b->q_level_off, loff.data(), loff.size() * 8, "queue levels")) ||
        (rc = upload(c, b->q_level_active, active.data(), active.size() * 4, "queue active")) ||
        (rc = upload(c, b->q_tile_prefix, prefix.data(), prefix.size() * 8, "queue prefix")) ||
        (rc = upload(c, b->q_order, b->order.data(), b->order.size() * 4, "queue order")) ||
        (rc = upload(c, b->sys_dev, b->sys.data(), b->sys.size() * sizeof(SysDev), "system table")))
        return rc;
    b->q.level_off = static_cast<const int64_t *>(b->q_level_off.p);
    b->q.level_active = static_cast<const int32_t *>(b->q_level_active.p);
    b->q.tile_prefix = static_cast<const int64_t *>(b->q_tile_prefix.p);
    b->q.order = static_cast<const int32_t *>(b->q_order.p);
    b->q.nlevels = b->nlevels;
    b->q.total = loff[b->nlevels];
    drop_graph(b);
    return CHEBTD_OK;
}

// Passes of the batched deep schedule for M orders at depth D: npass passes,
// the first next of them with D + 1 orders (D + 1 <= kMaxDepth), covering
// D npass + next <= M orders; the rest goes to two-order passes and the
// one-order tail.  The fewest passes that cover M exactly when there are
// such (P = ceil(M / (D + 1)) passes with P D <= M), else M / D passes taking
// one extra order each while orders are left.
void batch_deep_split(int M, int D, int *npass, int *next)
{
    const int E = D + 1 <= kMaxDepth ? D + 1 : 0;
    if (M < 1 || D < 1) {
        *npass = *next = 0;
    } else if (E && D * ((M + E - 1) / E) <= M) {
        *npass = (M + E - 1) / E;
        *next = M - D * *npass;
    } else {
        *npass = M / D;
        *next = E ? std::min(M - D * *npass, *npass) : 0;
    }
}

static hipError_t enqueue_step(Ctx *c, BatchState *b, hipStream_t s, int par)
{
    const SysDev *sys = static_cast<const SysDev *>(b->sys_dev.p);
    const double2 *gam = static_cast<const double2 *>(b->gamma_dev.p);
    if (b->mode == CHEBTD_SCHED_PAIRS) {
        const int32_t *ps = static_cast<const int32_t *>(b->pblk_sys.p);
        const int32_t *pw = static_cast<const int32_t *>(b->pblk_wave0.p);
        for (size_t p = 0; p < b->pair_level_blocks.size(); ++p) {
            hipError_t e = launch_batch_pair(s, sys, gam, ps, pw, b->pair_level_blocks[p], (int)p, 0, par);
            if (e != hipSuccess) return e;
        }
        return launch_batch_tail(s, sys, gam, static_cast<const int32_t *>(b->tblk_sys.p),
                                 static_cast<const int32_t *>(b->tblk_tile.p), b->ntail_blocks, b->tile, par,
                                 b->block, 0);
    }
    if (b->mode == CHEBTD_SCHED_DEEP) {
        const int32_t *dsys = static_cast<const int32_t *>(b->dblk_sys.p);
        const int32_t *dw = static_cast<const int32_t *>(b->dblk_wave0.p);
        const int D = b->deep_D;
        for (const auto &dl : b->deep_launches) {
            hipError_t e = launch_batch_deep(s, dl.depth, sys, gam, dsys + dl.off, dw + dl.off, dl.count, dl.pass, D,
                                             par);
            if (e != hipSuccess) return e;
        }
        const int32_t *ps = static_cast<const int32_t *>(b->dpblk_sys.p);
        const int32_t *pw = static_cast<const int32_t *>(b->dpblk_wave0.p);
        for (size_t q = 0; q + 1 < b->deep_pair_off.size(); ++q) {
            const int64_t o = b->deep_pair_off[q];
            hipError_t e = launch_batch_pair(s, sys, gam, ps + o, pw + o, b->deep_pair_off[q + 1] - o, (int)q, D,
                                             par);
            if (e != hipSuccess) return e;
        }
        return launch_batch_tail(s, sys, gam, static_cast<const int32_t *>(b->dtblk_sys.p),
                                 static_cast<const int32_t *>(b->dtblk_tile.p), b->ndtail_blocks, b->tile, par,
                                 b->block, 1);
    }
    if (b->mode == CHEBTD_SCHED_LEVELS) {
        for (int k = 0; k < b->nlevels; ++k) {
            hipError_t e = launch_batch_level(s, sys, gam, static_cast<const int32_t *>(b->blk_sys.p),
                                              static_cast<const int32_t *>(b->blk_tile.p), b->level_blocks[k],
                                              k, b->tile, par, b->block);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    const int64_t grid = std::min<int64_t>((int64_t)c->num_cus * b->wg_per_cu, b->q.total);
    return launch_batch_persistent(s, sys, gam, b->q, b->tile, par, static_cast<int64_t *>(b->head.p),
                                   static_cast<int32_t *>(b->done.p), static_cast<int32_t *>(b->flag.p),
                                   b->nsys, (int)std::max<int64_t>(grid, 1), b->block, b->spin_limit);
}

static int run_steps(Ctx *c, BatchState *b, int64_t K, bool use_graph)
{
    hipStream_t s = c->stream;
    hipError_t e = launch_batch_clear_flag(s, static_cast<int32_t *>(b->flag.p));
    if (e != hipSuccess) return hip_fail(c, e, "batch flag reset");
    if (use_graph && K >= 2) {
        if (!b->graph) {
            if (!b->cap) {
                e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
                if (e != hipSuccess) return hip_fail(c, e, "batch capture stream");
            }
            hipGraph_t g = nullptr;
            e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed);
            if (e != hipSuccess) return hip_fail(c, e, "batch capture");
            hipError_t e1 = enqueue_step(c, b, b->cap, 0);
            if (e1 == hipSuccess) e1 = enqueue_step(c, b, b->cap, 1);
            e = hipStreamEndCapture(b->cap, &g);
            if (e1 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return hip_fail(c, e1, "batch step capture");
            }
            if (e != hipSuccess) return hip_fail(c, e, "batch end capture");
            e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                b->graph = nullptr;
                return hip_fail(c, e, "batch graph instantiate");
            }
        }
        for (int64_t st = 0; st + 1 < K; st += 2) {
            e = hipGraphLaunch(b->graph, s);
            if (e != hipSuccess) return hip_fail(c, e, "batch graph launch");
        }
        if (K & 1) {
            e = enqueue_step(c, b, s, 0);
            if (e != hipSuccess) return hip_fail(c, e, "batch last step");
        }
    } else {
        for (int64_t st = 0; st < K; ++st) {
            e = enqueue_step(c, b, s, (int)(st & 1));
            if (e != hipSuccess) return hip_fail(c, e, "batch step");
        }
    }
    if (K & 1) {
        e = launch_batch_copy_back(s, static_cast<const SysDev *>(b->sys_dev.p),
                                   static_cast<const int32_t *>(b->blk_sys.p),
                                   static_cast<const int32_t *>(b->blk_tile.p), b->nblocks, b->tile, b->block);
        if (e != hipSuccess) return hip_fail(c, e, "batch copy back");
    }
    return CHEBTD_OK;
}

static int check_timeout(Ctx *c, BatchState *b)
{
    hipError_t e = hipMemcpyAsync(c->pinned, b->flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "batch completion");
    int32_t f = 0;
    std::memcpy(&f, c->pinned, sizeof(int32_t));
    if (f)
        return fail(c, CHEBTD_E_TIMEOUT,
                    "batch: a persistent workgroup's dependency wait ran out; results are invalid");
    return CHEBTD_OK;
}

static uint64_t shape_key(const Ctx *c, const BatchState *b)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (v >> (8 * i)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    mix((uint64_t)b->nsys);
    mix((uint64_t)c->num_cus);
    for (int s = 0; s < b->nsys; ++s) {
        mix((uint64_t)b->sys[s].W);
        mix((uint64_t)b->sys[s].L);
        mix((uint64_t)b->sys[s].edge);
        mix((uint64_t)b->M[s]);
    }
    return h;
}

}  // namespace chebtd

using namespace chebtd;
struct chebtd_ctx : public Ctx {};

extern "C" {

int chebtd_batch_create(chebtd_ctx *ctx, int nsys, const chebtd_sys_desc *descs, double dt, double alpha,
                        double tol)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = static_cast<Ctx *>(ctx);
    if (nsys < 1 || !descs || !(dt >= 0.0) || !std::isfinite(dt) || !(alpha >= 0.0))
        return fail(c, CHEBTD_E_ARG, "chebtd_batch_create: need nsys >= 1, descriptors, dt >= 0, alpha >= 0");
    if (!(tol > 0.0)) tol = 1e-15;
    for (int s = 0; s < nsys; ++s) {
        const chebtd_sys_desc &d = descs[s];
        if (d.width < 1 || d.length < 1 || d.width * d.length >= ((int64_t)1 << 31) || !d.eps_dev ||
            !d.psi_dev || (d.edge != CHEBTD_ZIGZAG && d.edge != CHEBTD_ARMCHAIR) || !(d.emax > d.emin) ||
            !std::isfinite(d.emin) || !std::isfinite(d.emax) || !std::isfinite(d.t_hop))
            return fail(c, CHEBTD_E_ARG, "chebtd_batch_create: bad descriptor " + std::to_string(s));
    }
    batch_destroy(c);
    BatchState *b = new (std::nothrow) BatchState();
    if (!b) return fail(c, CHEBTD_E_OOM, "batch state");
    c->batch = b;
    b->nsys = nsys;
    b->dt = dt;
    {
        // two seconds of the device's constant-rate wall clock
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) != hipSuccess || khz <= 0)
            khz = 100000;
        b->spin_limit = (int64_t)khz * 1000 * 2;
    }
    b->sys.resize(nsys);
    b->M.resize(nsys);
    b->nsites.resize(nsys);
    int64_t total = 0;
    std::vector<double> g;
    for (int s = 0; s < nsys; ++s) {
        const chebtd_sys_desc &d = descs[s];
        double a = 0, bb = 0;
        shift_scale(d.emin, d.emax, alpha, &a, &bb);
        const int M = truncation_order(a * dt, tol);
        if (M < 0) {
            batch_destroy(c);
            return fail(c, CHEBTD_E_ARG, "chebtd_batch_create: bad a*dt for system " + std::to_string(s));
        }
        step_weights(a, bb, dt, M, g);
        SysDev &sd = b->sys[s];
        sd.eps = d.eps_dev;
        sd.psi = reinterpret_cast<double2 *>(d.psi_dev);
        sd.W = (int32_t)d.width;
        sd.L = (int32_t)d.length;
        sd.edge = d.edge;
        sd.M = M;
        sd.b = bb;
        sd.s2 = 2.0 / a;
        sd.off2 = -2.0 * d.t_hop / a;
        sd.gamma_off = (int64_t)b->gamma.size() / 2;
        b->gamma.insert(b->gamma.end(), g.begin(), g.end());
        b->M[s] = M;
        b->nsites[s] = d.width * d.length;
        total += b->nsites[s];
    }
    int rc = ensure(c, b->work, (size_t)total * 4 * sizeof(double2), "batch work vectors");
    if (rc) {
        batch_destroy(c);
        return rc;
    }
    double2 *w = static_cast<double2 *>(b->work.p);
    b->pairs_ok = true;
    for (int s = 0; s < nsys; ++s) {
        SysDev &sd = b->sys[s];
        sd.A = w;
        sd.B = w + b->nsites[s];
        sd.C = w + 2 * b->nsites[s];
        sd.D = w + 3 * b->nsites[s];
        w += 4 * b->nsites[s];
        sd.rows = pair_rows_for_width(sd.W);
        sd.nstrips = (sd.L + kPairStripCols - 1) / kPairStripCols;
        sd.nchunks = (sd.W + sd.rows - 1) / sd.rows;
        sd.pad2 = 0;
        if (b->M[s] < 2) b->pairs_ok = false;  // the head of a pair level computes two orders
        sd.npass_pairs = b->M[s] >> 1;
    }
    // deep schedule: passes of D = deep_D (CHEBTD_BATCH_DEPTH, 4 .. 6,
    // overrides) or D + 1 orders, so every system needs M >= D.  On these
    // HBM-bound passes a pass costs about the same whatever its depth
    // (measured on MI355X over the 256-ribbon workload: 1020, 1024 and 1062
    // us for four, five and six orders; a two-order pass 1042 us over the
    // same systems), so each system takes the fewest passes: P = ceil(M /
    // (D + 1)) of them when P D <= M (M - P D of them with D + 1 orders),
    // else M / D passes that take up to one extra order each, with pairs and
    // the tail for what is left.  Chunk heights as for one ribbon below 4M
    // sites (the systems here are far smaller; on the 256-ribbon workload
    // over 200 steps 10 rows ran 211 G site-orders/s, 16 rows 209 G, 22 rows
    // 205 G); CHEBTD_BATCH_DEEP_ROWS overrides
    if (const char *env = std::getenv("CHEBTD_BATCH_DEPTH")) b->deep_D = std::max(4, std::min(6, std::atoi(env)));
    b->deep_ok = b->pairs_ok;
    static const int drows_of[7] = {0, 0, 0, 8, 6, 10, 14};
    int drows_env = 0;
    if (const char *env = std::getenv("CHEBTD_BATCH_DEEP_ROWS")) drows_env = std::max(1, std::atoi(env));
    for (int s = 0; s < nsys; ++s) {
        SysDev &sd = b->sys[s];
        const int D = b->deep_D, E = D + 1 <= kMaxDepth ? D + 1 : 0, M = b->M[s];
        if (M < D || !deep_offsets_fit(sd.W, sd.L)) b->deep_ok = false;
        sd.drows = std::min<int32_t>(sd.W, drows_env ? drows_env : drows_of[D]);
        sd.dnstrips = (sd.L + deep_strip_cols(D) - 1) / deep_strip_cols(D);
        sd.dnchunks = (sd.W + sd.drows - 1) / sd.drows;
        sd.drows_ext = E ? std::min<int32_t>(sd.W, drows_env ? drows_env : drows_of[E]) : sd.drows;
        sd.dnstrips_ext = E ? (sd.L + deep_strip_cols(E) - 1) / deep_strip_cols(E) : sd.dnstrips;
        sd.dnchunks_ext = (sd.W + sd.drows_ext - 1) / sd.drows_ext;
        int npass = 0, next = 0;  // passes, of which with D + 1 orders
        batch_deep_split(M, D, &npass, &next);
        sd.ndeep = npass;
        sd.ndeep_ext = next;
        sd.kdeep = D * npass + next;
        sd.npass_deep = sd.ndeep + (M - sd.kdeep) / 2;
    }
    b->order.resize(nsys);
    for (int s = 0; s < nsys; ++s) b->order[s] = s;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int32_t x, int32_t y) { return b->M[x] > b->M[y]; });
    if ((rc = upload(c, b->gamma_dev, b->gamma.data(), b->gamma.size() * sizeof(double), "batch weights")) ||
        (rc = ensure(c, b->head, sizeof(int64_t), "queue head")) ||
        (rc = ensure(c, b->done, (size_t)nsys * sizeof(int32_t), "completion counters")) ||
        (rc = ensure(c, b->flag, sizeof(int32_t), "timeout flag")) || (rc = build_tables(c, b))) {
        batch_destroy(c);
        return rc;
    }
    return CHEBTD_OK;
}

int chebtd_batch_set_schedule(chebtd_ctx *ctx, int mode, int tile_rows, int block, int wg_per_cu)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = static_cast<Ctx *>(ctx);
    BatchState *b = c->batch;
    if (!b) return fail(c, CHEBTD_E_STATE, "chebtd_batch_set_schedule: no batch");
    if (mode == CHEBTD_SCHED_PAIRS && !b->pairs_ok)
        return fail(c, CHEBTD_E_ARG, "chebtd_batch_set_schedule: the pairs schedule needs M >= 2 for every system");
    if (mode == CHEBTD_SCHED_DEEP && !b->deep_ok)
        return fail(c, CHEBTD_E_ARG,
                    "chebtd_batch_set_schedule: the deep schedule needs M >= its depth for every system and "
                    "ribbons whose offsets fit 32 bits");
    if ((mode != CHEBTD_SCHED_LEVELS && mode != CHEBTD_SCHED_PERSISTENT && mode != CHEBTD_SCHED_PAIRS &&
         mode != CHEBTD_SCHED_DEEP) ||
        block < 64 || block > 1024 ||
        block % 64 || tile_rows < block || tile_rows % block || wg_per_cu < 1 || wg_per_cu > 8)
        return fail(c, CHEBTD_E_ARG,
                    "chebtd_batch_set_schedule: need a known mode, block in [64,1024] (multiple of 64), "
                    "tile_rows a multiple of block, 1 <= wg_per_cu <= 8");
    const bool retile = tile_rows != b->tile;
    b->mode = mode;
    b->tile = tile_rows;
    b->block = block;
    b->wg_per_cu = wg_per_cu;
    drop_graph(b);
    return retile ? build_tables(c, b) : CHEBTD_OK;
}

// Point the systems at new states: the kernels (and a captured graph) read
// psi from the device system table, so an upload of the table on the stream
// re-binds them for every later launch.
static int rebind_states(Ctx *c, BatchState *b, double *const *psi_dev)
{
    bool same = true;
    for (int s = 0; s < b->nsys; ++s) {
        if (!psi_dev[s]) return fail(c, CHEBTD_E_ARG, "chebtd_batch_propagate: null state of system " +
                                                          std::to_string(s));
        same = same && reinterpret_cast<double2 *>(psi_dev[s]) == b->sys[s].psi;
    }
    if (same) return CHEBTD_OK;
    const size_t bytes = b->sys.size() * sizeof(SysDev);
    hipError_t e = hipSuccess;
    if (!b->sys_pinned) {
        e = hipHostMalloc(reinterpret_cast<void **>(&b->sys_pinned), bytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            b->sys_pinned = nullptr;
            return fail(c, CHEBTD_E_OOM, "chebtd_batch_propagate: pinned system table");
        }
        e = hipEventCreateWithFlags(&b->sys_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            b->sys_ev = nullptr;
            return hip_fail(c, e, "chebtd_batch_propagate: event");
        }
    }
    // the previous upload may still be reading the mirror
    if (b->sys_ev_pending && (e = hipEventSynchronize(b->sys_ev)) != hipSuccess)
        return hip_fail(c, e, "chebtd_batch_propagate: previous table upload");
    for (int s = 0; s < b->nsys; ++s) b->sys[s].psi = reinterpret_cast<double2 *>(psi_dev[s]);
    std::memcpy(b->sys_pinned, b->sys.data(), bytes);
    e = hipMemcpyAsync(b->sys_dev.p, b->sys_pinned, bytes, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipEventRecord(b->sys_ev, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "chebtd_batch_propagate: table upload");
    b->sys_ev_pending = true;
    return CHEBTD_OK;
}

int chebtd_batch_propagate(chebtd_ctx *ctx, double *const *psi_dev, int64_t K, unsigned flags)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = static_cast<Ctx *>(ctx);
    BatchState *b = c->batch;
    if (!b) return fail(c, CHEBTD_E_STATE, "chebtd_batch_propagate: no batch");
    if (K < 0) return fail(c, CHEBTD_E_ARG, "chebtd_batch_propagate: K < 0");
    if (psi_dev) {
        const int rc = rebind_states(c, b, psi_dev);
        if (rc) return rc;
    }
    if (K == 0) return CHEBTD_OK;
    int rc = run_steps(c, b, K, (flags & CHEBTD_GRAPH) != 0);
    if (rc) return rc;
    if (flags & CHEBTD_NO_CHECK) return CHEBTD_OK;
    return check_timeout(c, b);
}

int chebtd_batch_info(const chebtd_ctx *ctx, int *nsys, int *M_host)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    const Ctx *c = static_cast<const Ctx *>(ctx);
    if (!c->batch) return fail(const_cast<Ctx *>(c), CHEBTD_E_STATE, "chebtd_batch_info: no batch");
    if (nsys) *nsys = c->batch->nsys;
    if (M_host)
        for (int s = 0; s < c->batch->nsys; ++s) M_host[s] = c->batch->M[s];
    return CHEBTD_OK;
}

int chebtd_batch_autotune(chebtd_ctx *ctx, const char *cache_path, int *best_out)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = static_cast<Ctx *>(ctx);
    BatchState *b = c->batch;
    if (!b) return fail(c, CHEBTD_E_STATE, "chebtd_batch_autotune: no batch");
    const uint64_t key = shape_key(c, b);
    char keystr[32];
    std::snprintf(keystr, sizeof keystr, "%016llx", (unsigned long long)key);
    int best[4] = {-1, 0, 0, 0};
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k;
            int m, t, bl, w;
            if ((ls >> k >> m >> t >> bl >> w) && k == keystr) {
                best[0] = m;
                best[1] = t;
                best[2] = bl;
                best[3] = w;
            }
        }
    }
    if (best[0] < 0) {
        // save every system's state, time each candidate on the real batch, restore
        int64_t total = 0;
        for (int s = 0; s < b->nsys; ++s) total += b->nsites[s];
        DevBuf save;
        int rc = ensure(c, save, (size_t)total * sizeof(double2), "autotune backup");
        if (rc) return rc;
        hipStream_t s = c->stream;
        auto copy_all = [&](bool to_save) -> hipError_t {
            double2 *p = static_cast<double2 *>(save.p);
            for (int q = 0; q < b->nsys; ++q) {
                const size_t bytes = (size_t)b->nsites[q] * sizeof(double2);
                hipError_t e = to_save ? hipMemcpyAsync(p, b->sys[q].psi, bytes, hipMemcpyDeviceToDevice, s)
                                       : hipMemcpyAsync(b->sys[q].psi, p, bytes, hipMemcpyDeviceToDevice, s);
                if (e != hipSuccess) return e;
                p += b->nsites[q];
            }
            return hipSuccess;
        };
        hipError_t e = copy_all(true);
        if (e != hipSuccess) {
            release(save);
            return hip_fail(c, e, "autotune backup");
        }
        struct Cand {
            int mode, tile, block, wg;
        };
        // per-launch schedules first; the persistent ones last, dropped once
        // one of them takes more than twice the best time so far
        std::vector<Cand> cands;
        for (int tile : {1024, 2048, 4096, 8192})
            for (int block : {256, 512}) {
                if (tile % block) continue;
                if (b->deep_ok) cands.push_back({CHEBTD_SCHED_DEEP, tile, block, 1});
                if (b->pairs_ok) cands.push_back({CHEBTD_SCHED_PAIRS, tile, block, 1});
                cands.push_back({CHEBTD_SCHED_LEVELS, tile, block, 1});
            }
        for (int tile : {1024, 2048, 4096, 8192})
            for (int block : {256, 512})
                if (tile % block == 0)
                    for (int wg : {2, 4}) cands.push_back({CHEBTD_SCHED_PERSISTENT, tile, block, wg});
        double best_ms = 1e300;
        for (const Cand &cd : cands) {
            // a candidate that fails its own way (refused, or a persistent
            // schedule whose dependency wait ran out) is skipped; a HIP
            // failure ends the search.  The states are restored either way.
            rc = chebtd_batch_set_schedule(ctx, cd.mode, cd.tile, cd.block, cd.wg);
            if (!rc) rc = run_steps(c, b, 1, false);  // warm-up
            if (!rc) rc = check_timeout(c, b);
            float ms = 0.f;
            if (!rc) {
                e = hipEventRecord(c->ev_a, s);
                if (e == hipSuccess) rc = run_steps(c, b, 2, false);
                if (e == hipSuccess && !rc) e = hipEventRecord(c->ev_b, s);
                if (e == hipSuccess && !rc) e = hipEventSynchronize(c->ev_b);
                if (e == hipSuccess && !rc) e = hipEventElapsedTime(&ms, c->ev_a, c->ev_b);
                if (e != hipSuccess) rc = hip_fail(c, e, "autotune timing");
                if (!rc) rc = check_timeout(c, b);
            }
            const hipError_t er = copy_all(false);
            if (er != hipSuccess) {
                rc = hip_fail(c, er, "autotune restore");
                break;
            }
            if (rc == CHEBTD_E_ARG || rc == CHEBTD_E_TIMEOUT) {
                rc = CHEBTD_OK;
                continue;
            }
            if (rc) break;
            const bool slow_persistent = cd.mode == CHEBTD_SCHED_PERSISTENT && ms > 2.0 * best_ms;
            if (ms < best_ms) {
                best_ms = ms;
                best[0] = cd.mode;
                best[1] = cd.tile;
                best[2] = cd.block;
                best[3] = cd.wg;
            }
            if (slow_persistent) break;
        }
        {
            // every exit restores the caller's states before the backup goes
            e = copy_all(false);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess && !rc) rc = hip_fail(c, e, "autotune restore");
        }
        release(save);
        if (rc) return rc;
        if (best[0] < 0) return fail(c, CHEBTD_E_ARG, "chebtd_batch_autotune: no schedule ran on this batch");
        if (cache_path) {
            std::ofstream out(cache_path, std::ios::app);
            out << keystr << ' ' << best[0] << ' ' << best[1] << ' ' << best[2] << ' ' << best[3] << '\n';
        }
    }
    int rc = chebtd_batch_set_schedule(ctx, best[0], best[1], best[2], best[3]);
    if (rc) return rc;
    if (best_out)
        for (int i = 0; i < 4; ++i) best_out[i] = best[i];
    return CHEBTD_OK;
}

}  // extern "C"
