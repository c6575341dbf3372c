// Host builder of the generalised Holstein Hamiltonian, eq. (ghm) of
// arXiv:0907.3022 (Sect. 3.3): one spinless electron on L sites times phonon
// Fock states with at most nph phonons in total.
//
// Phonon configurations are ranked in closed form with the combinatorial
// number system: configurations of total T start at C(T-1+L, L) (all
// configurations of smaller total), and inside one total the order is
// lexicographic ascending in (n_1..n_L).  The rank of n is that offset plus,
// for every position j before the last, the number of compositions that
// agree on n_1..n_{j-1} and have a smaller value at j:
//   C(r_j + m_j, m_j) - C(r_j - n_j + m_j, m_j),
// with r_j the phonons left for positions j..L and m_j = L - j parts after j.
#include <algorithm>
#include <thread>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace chebtd {

namespace {

struct Binom {
    int nmax = 0, kmax = 0;
    std::vector<int64_t> t;
    bool ok = true;
    Binom(int nmax_, int kmax_) : nmax(nmax_), kmax(kmax_), t((size_t)(nmax_ + 1) * (kmax_ + 1), 0)
    {
        for (int n = 0; n <= nmax; ++n) {
            at(n, 0) = 1;
            for (int k = 1; k <= std::min(n, kmax); ++k) {
                int64_t a = at(n - 1, k - 1), b = (k <= n - 1) ? at(n - 1, k) : 0;
                if (a > INT64_MAX - b) ok = false;
                at(n, k) = a + b;
            }
        }
    }
    int64_t &at(int n, int k) { return t[(size_t)n * (kmax + 1) + k]; }
    int64_t operator()(int n, int k) const
    {
        if (k < 0 || n < 0 || k > n) return 0;
        return t[(size_t)n * (kmax + 1) + k];
    }
};

int64_t rank_of(const Binom &C, const uint8_t *n, int L)
{
    int T = 0;
    for (int j = 0; j < L; ++j) T += n[j];
    int64_t r = (T == 0) ? 0 : C(T - 1 + L, L);
    int left = T;
    for (int j = 0; j + 1 < L; ++j) {
        const int m = L - 1 - j;
        r += C(left + m, m) - C(left - n[j] + m, m);
        left -= n[j];
    }
    return r;
}

// Next configuration in basis order; returns false after the last one.
bool next_config(uint8_t *n, int L, int nph)
{
    int T = 0;
    for (int j = 0; j < L; ++j) T += n[j];
    // rightmost position j <= L-2 whose prefix sum is still below T
    int prefix = T - n[L - 1];
    for (int j = L - 2; j >= 0; --j) {
        if (prefix < T) {
            n[j]++;
            int s = 0;
            for (int q = 0; q <= j; ++q) s += n[q];
            for (int q = j + 1; q < L - 1; ++q) n[q] = 0;
            n[L - 1] = (uint8_t)(T - s);
            return true;
        }
        prefix -= n[j];
    }
    if (T >= nph) return false;
    std::memset(n, 0, (size_t)L);
    n[L - 1] = (uint8_t)(T + 1);
    return true;
}

// Configuration of rank `r` (inverse of rank_of).
void unrank(const Binom &C, int64_t r, uint8_t *n, int L, int nph)
{
    int T = 0;
    while (T < nph && C(T + L, L) <= r) ++T;  // C(T+L, L) = configurations of total <= T
    int64_t within = r - (T == 0 ? 0 : C(T - 1 + L, L));
    int left = T;
    for (int j = 0; j + 1 < L; ++j) {
        const int m = L - 1 - j;
        const int64_t all = C(left + m, m);
        int v = 0;
        // largest v whose preceding count fits in `within`
        while (v < left && all - C(left - (v + 1) + m, m) <= within) ++v;
        within -= all - C(left - v + m, m);
        n[j] = (uint8_t)v;
        left -= v;
    }
    n[L - 1] = (uint8_t)left;
}

}  // namespace

int holstein_tables(int L, int nph, int periodic, HolsteinTables &out, std::string &err)
{
    if (L < 1 || L > 64 || nph < 0 || nph > 254) {
        err = "holstein: need 1 <= L <= 64 and 0 <= nph <= 254";
        return CHEBTD_E_ARG;
    }
    if (periodic && L < 3) {
        err = "holstein: a ring needs L >= 3";
        return CHEBTD_E_ARG;
    }
    Binom C(L + nph + 1, L);
    if (!C.ok) {
        err = "holstein: basis too large";
        return CHEBTD_E_ARG;
    }
    const int64_t nconf = C(L + nph, L);
    const int64_t n = nconf * (int64_t)L;
    if (n >= (int64_t)INT32_MAX) {
        err = "holstein: dimension exceeds 2^31 - 1";
        return CHEBTD_E_ARG;
    }
    out.L = L;
    out.nph = nph;
    out.nconf = nconf;
    out.n = n;
    out.up.assign((size_t)n, -1);
    out.dn.assign((size_t)n, -1);
    out.occ.assign((size_t)n, 0);
    out.tot.assign((size_t)nconf, 0);
    // configurations are independent: split the rank range over host threads
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (nconf < 4096) nt = 1;
    std::vector<std::thread> pool;
    for (unsigned tix = 0; tix < nt; ++tix) {
        const int64_t r0 = nconf * tix / nt, r1 = nconf * (tix + 1) / nt;
        pool.emplace_back([&, r0, r1]() {
            std::vector<uint8_t> cfg((size_t)L), tmp((size_t)L);
            if (r0 >= r1) return;
            unrank(C, r0, cfg.data(), L, nph);
            for (int64_t r = r0; r < r1; ++r) {
                int T = 0;
                for (int j = 0; j < L; ++j) T += cfg[(size_t)j];
                out.tot[(size_t)r] = (uint8_t)T;
                for (int i = 0; i < L; ++i) {
                    const size_t row = (size_t)i * (size_t)nconf + (size_t)r;
                    out.occ[row] = cfg[(size_t)i];
                    if (T < nph) {
                        tmp = cfg;
                        tmp[(size_t)i]++;
                        out.up[row] = (int32_t)rank_of(C, tmp.data(), L);
                    }
                    if (cfg[(size_t)i] > 0) {
                        tmp = cfg;
                        tmp[(size_t)i]--;
                        out.dn[row] = (int32_t)rank_of(C, tmp.data(), L);
                    }
                }
                if (r + 1 < r1) next_config(cfg.data(), L, nph);
            }
        });
    }
    for (auto &th : pool) th.join();
    return CHEBTD_OK;
}

int holstein_count(int L, int nph, int64_t *count)
{
    if (L < 1 || nph < 0 || nph > 255 || L > 64) return -1;
    Binom C(L + nph, L);
    if (!C.ok) return -1;
    *count = C(L + nph, L);
    return 0;
}

int holstein_build(int L, int nph, double t, double w0, const double *g, const double *Delta,
                   int periodic, HolsteinCsr &out, std::string &err)
{
    if (!g || !Delta) {
        err = "holstein: g and Delta must be non-null";
        return CHEBTD_E_ARG;
    }
    HolsteinTables tb;
    const int rc = holstein_tables(L, nph, periodic, tb, err);
    if (rc) return rc;
    const int64_t C = tb.nconf, n = tb.n;
    out.n = n;
    out.nconf = C;
    out.rowptr.assign((size_t)n + 1, 0);
    out.col.clear();
    out.val.clear();
    out.col.reserve((size_t)n * 5);
    out.val.reserve((size_t)n * 10);
    struct Entry {
        int64_t c;
        double v;
    };
    Entry row[5];
    // rows in state order: site-major, configurations by rank within a site
    for (int i = 0; i < L; ++i) {
        int lft = i - 1, rgt = i + 1;
        if (periodic) {
            lft = (i + L - 1) % L;
            rgt = (i + 1) % L;
        }
        for (int64_t r = 0; r < C; ++r) {
            const int64_t s = (int64_t)i * C + r;
            const int T = tb.tot[(size_t)r];
            const int ni = tb.occ[(size_t)s];
            int cnt = 0;
            row[cnt++] = {s, Delta[i] + w0 * T};
            if (lft >= 0) row[cnt++] = {(int64_t)lft * C + r, -t};
            if (rgt < L) row[cnt++] = {(int64_t)rgt * C + r, -t};
            if (tb.up[(size_t)s] >= 0)
                row[cnt++] = {(int64_t)i * C + tb.up[(size_t)s], -g[i] * w0 * std::sqrt((double)ni + 1.0)};
            if (tb.dn[(size_t)s] >= 0)
                row[cnt++] = {(int64_t)i * C + tb.dn[(size_t)s], -g[i] * w0 * std::sqrt((double)ni)};
            std::sort(row, row + cnt, [](const Entry &x, const Entry &y) { return x.c < y.c; });
            for (int q = 0; q < cnt; ++q) {
                out.col.push_back((int32_t)row[q].c);
                out.val.push_back(row[q].v);
                out.val.push_back(0.0);
            }
            out.rowptr[(size_t)s + 1] = (int64_t)out.col.size();
        }
    }
    out.nnz = (int64_t)out.col.size();
    return CHEBTD_OK;
}

}  // namespace chebtd
