// Host-side exercise of the library's runtime for the sanitizer build of the
// tests: the plan helpers (Bessel values by Miller's backward recurrence,
// truncation order, weights of eq. (U_1)), the Holstein basis tables and CSR
// builder of eq. (ghm) (threaded), the argument checks of the C ABI entry
// points, the batched schedule's split of M into passes and the shapes of
// the several-workgroup chain run, none of which needs a GPU.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer (host code only); any report aborts the run.
// Exit status 0: every check passed.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "batch_internal.h"
#include "chebtd.h"
#include "internal.h"

namespace chebtd {
std::vector<int> plan_passes(const Ctx &c, int M);  // api.cpp
}

using namespace chebtd;

static int failures = 0;
#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

int main()
{
    // plan helpers over eleven decades of a*dt, zero included
    for (int e = -14; e <= 8; ++e) {
        for (double m : {1.0, 3.7}) {
            const double z = e == -14 ? 0.0 : m * std::pow(10.0, 0.5 * e);
            const int M = truncation_order(z, 1e-15);
            CHECK(M >= 0);
            std::vector<double> J;
            CHECK(bessel_miller(z, M + 8, J) == 0);
            CHECK((int)J.size() >= M + 9);
            double s = J[0];
            for (size_t k = 2; k < J.size(); k += 2) s += 2.0 * J[k];
            CHECK(std::fabs(s - 1.0) < 1e-9);
            std::vector<double> g;
            double a = 0.0, b = 0.0;
            shift_scale(-3.0, 5.0, 0.01, &a, &b);
            step_weights(a, b, z / a, M, g);
            CHECK((int)g.size() == 2 * (M + 1));
        }
    }
    // Holstein tables and CSR, rings and open chains; the larger ones split
    // the basis over host threads
    const int shapes[][3] = {{1, 6, 0}, {2, 5, 0}, {3, 4, 1}, {5, 3, 1}, {7, 9, 0}, {10, 6, 1}, {12, 5, 0}};
    for (const auto &sh : shapes) {
        const int L = sh[0], nph = sh[1], per = sh[2];
        HolsteinTables t;
        std::string err;
        CHECK(holstein_tables(L, nph, per, t, err) == 0);
        int64_t cnt = 0;
        CHECK(holstein_count(L, nph, &cnt) == 0);
        CHECK(t.nconf == cnt && t.n == cnt * L);
        std::vector<double> g(L, 0.7), D(L, 0.1);
        HolsteinCsr h;
        CHECK(holstein_build(L, nph, 1.0, 1.3, g.data(), D.data(), per, h, err) == 0);
        CHECK(h.n == t.n && (int64_t)h.rowptr.size() == h.n + 1 && h.rowptr.back() == h.nnz);
        for (int64_t i = 0; i < t.n; ++i) {
            CHECK(t.up[(size_t)i] < (int32_t)t.nconf && t.dn[(size_t)i] < (int32_t)t.nconf);
            if (failures > 20) break;
        }
    }
    {
        HolsteinTables t;
        std::string err;
        CHECK(holstein_tables(2, 3, 1, t, err) != 0);  // a ring needs three sites
        CHECK(holstein_tables(0, 3, 0, t, err) != 0);
    }
    // argument checks of the C ABI (no GPU is touched)
    double d = 0.0;
    int64_t r = 0;
    CHECK(chebtd_h_chain1d(nullptr, 10, 0.1, &d) == CHEBTD_E_ARG);
    CHECK(chebtd_plan(nullptr, 1.0, 1e-15, nullptr) == CHEBTD_E_ARG);
    CHECK(chebtd_propagate(nullptr, &d, 1, nullptr, nullptr, 0) == CHEBTD_E_ARG);
    CHECK(chebtd_adjoint_run(nullptr, 1, &d, &d) == CHEBTD_E_ARG);
    CHECK(chebtd_checkpoint_run(nullptr, &r) == CHEBTD_E_ARG);
    CHECK(chebtd_batch_propagate(nullptr, nullptr, 1, 0) == CHEBTD_E_ARG);
    CHECK(chebtd_batch_create(nullptr, 1, nullptr, 1.0, 0.01, 1e-15) == CHEBTD_E_ARG);
    CHECK(chebtd_create(nullptr, nullptr) == CHEBTD_E_ARG);
    CHECK(chebtd_last_error(nullptr) != nullptr);
    CHECK(chebtd_destroy(nullptr) == CHEBTD_OK);
    int64_t n = 0, nnz = 0;
    CHECK(chebtd_holstein_csr_host(2, 3, 1.0, 1.0, &d, &d, 1, &n, &nnz, nullptr, nullptr, nullptr) != CHEBTD_OK);
    // the batched deep schedule's passes: they cover M with at most one
    // extra order per pass, the fewest passes whenever passes of D and D + 1
    // orders can cover M exactly, and (D = 5) the single-system plan's split
    // of the same M on a small ribbon from 10 orders on
    Ctx rib;
    rib.kind = HKind::Honeycomb;
    rib.W = 16;
    rib.L = 64;
    rib.n = rib.W * rib.L;
    for (int D = 4; D <= 6; ++D)
        for (int M = D; M <= 300; ++M) {
            int np = -1, ne = -1;
            batch_deep_split(M, D, &np, &ne);
            const int kdeep = D * np + ne, rest = M - kdeep;
            CHECK(np >= 1 && ne >= 0 && ne <= np && rest >= 0 && rest < D);
            CHECK(ne == 0 || D + 1 <= kMaxDepth);
            const int P = D + 1 <= kMaxDepth ? (M + D) / (D + 1) : 0;
            if (P && D * P <= M) CHECK(rest == 0 && np == P);
            if (D == 5 && M >= 10) {
                std::vector<int> want(ne, D + 1);
                want.insert(want.end(), np - ne, D);
                want.insert(want.end(), rest / 2, 2);
                if (rest & 1) want.push_back(1);
                CHECK(plan_passes(rib, M) == want);
            }
        }
    // the several-workgroup chain run's shapes: every chain site owned by
    // exactly one workgroup, strips inside the own sites, halo depth even
    // and at most a third of a workgroup's sites, the epoch ring deep
    // enough, the scratch sized for the strips; one workgroup otherwise
    for (int64_t n = 1; n <= 4200; ++n) {
        const ChainMultiCfg cfg = chain_multi_config(n);
        if (cfg.R == 0) {
            CHECK(n <= 128 || n > 4096);
            CHECK(chain_multi_scratch_bytes(cfg) == 0);
            continue;
        }
        CHECK(n > 128 && n <= 4096 && cfg.T == 64);
        CHECK((int64_t)cfg.R * cfg.T == cfg.S + 2 * cfg.H && cfg.S >= cfg.H && cfg.H >= 2 && cfg.H % 2 == 0);
        CHECK(cfg.P >= 2 && cfg.P <= kChainMaxWG && kChainRing >= cfg.P + 1);
        CHECK(cfg.P * cfg.S >= n && (cfg.P - 1) * cfg.S < n);
        CHECK(chain_multi_scratch_bytes(cfg) >= (size_t)2 * cfg.P * 4 * cfg.H * 16);
    }
    std::printf("host_check: %d failures\n", failures);
    return failures == 0 ? 0 : 1;
}
