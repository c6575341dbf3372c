/*
 * Serial CPU reference ("oracle") for Chebyshev time propagation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the test-suite, the package's smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no code, header, table or
 * constant generator with the GPU path.
 *
 * Method: H. Fehske, J. Schleede, G. Schubert, G. Wellein, V. S. Filinov,
 * A. R. Bishop, "Numerical approaches to time evolution of complex quantum
 * systems" (arXiv:0907.3022).  Section 2.2 ("Chebyshev scheme"), eq. (U_1),
 * the Bessel form of c_k, the three-term recursion and the truncation rule
 * eq. (dec_Bessel); Crank-Nicolson eq. (CN) with the Thomas algorithm
 * (Sect. 3.2); the models of Sect. 3.1 (double well), eq. (model)
 * (honeycomb ribbon) and eq. (ghm) (Holstein polaron).
 *
 * Everything is plain fp64 with C99 complex numbers and straightforward
 * loops: every Hamiltonian is assembled as an explicit CSR matrix and applied
 * row by row, in the order the paper states the algorithm.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *  - extreme eigenvalues: Gershgorin discs;
 *  - truncation: M = (first k > z with |J_k(z)| < tol) - 1;
 *  - Bessel values: Miller's backward recurrence normalised by
 *    J_0 + 2 sum_k J_2k = 1;
 *  - hbar = 1 throughout.
 *
 * Parity-pinned by the CPU tests (closed forms, dense exact diagonalisation,
 * library Bessel values, brute force); no function here is "parity unpinned".
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Bessel functions of the first kind, integer order (coefficients c_k,      */
/* Sect. 2.2: c_k(z) = (-i)^k J_k(z)).                                       */
/* Miller's backward recurrence J_{k-1} = (2k/z) J_k - J_{k+1}, started far  */
/* beyond max(kmax, z) where J is negligible, then normalised with the       */
/* Neumann sum J_0 + 2 sum_{k>=1} J_{2k} = 1.  Values are rescaled whenever   */
/* they exceed 1e250 so the recurrence never overflows.                      */
/* Returns 0 on success, -1 on bad arguments.                                */
/* ------------------------------------------------------------------------ */
int orc_bessel_j(double z, int kmax, double *J)
{
    if (kmax < 0 || !J || !(z >= 0.0) || !isfinite(z)) return -1;
    if (z == 0.0) {
        J[0] = 1.0;
        for (int k = 1; k <= kmax; ++k) J[k] = 0.0;
        return 0;
    }
    if (z < 1e-8) {
        /* leading terms of the power series J_k(z) = (z/2)^k / k! (1 - ...) */
        double term = 1.0;
        for (int k = 0; k <= kmax; ++k) {
            if (k > 0) term *= (0.5 * z) / k;
            J[k] = term * (1.0 - 0.25 * z * z / (k + 1));
        }
        return 0;
    }
    int n0 = kmax > (int)ceil(z) ? kmax : (int)ceil(z);
    int ks = n0 + 40 + (int)sqrt(60.0 * n0);
    if (ks % 2) ks += 1; /* even start so the Neumann sum pairs up cleanly */

    double *w = (double *)calloc((size_t)ks + 2, sizeof(double));
    if (!w) return -1;
    w[ks + 1] = 0.0;
    w[ks] = 1e-300;
    for (int k = ks; k >= 1; --k) {
        w[k - 1] = (2.0 * k / z) * w[k] - w[k + 1];
        if (fabs(w[k - 1]) > 1e250) {
            for (int j = k - 1; j <= ks + 1; ++j) w[j] *= 1e-250;
        }
    }
    double norm = w[0];
    for (int k = 2; k <= ks; k += 2) norm += 2.0 * w[k];
    for (int k = 0; k <= kmax; ++k) J[k] = w[k] / norm;
    free(w);
    return 0;
}

/* Truncation order (Sect. 2.2, eq. (dec_Bessel)): the smallest M such that
 * every |c_k| = |J_k(z)| with k > M lies below tol.  J_k(z) decreases
 * monotonically for k > z, so M + 1 is the first k > z with |J_k| < tol.
 * Returns M >= 0, or -1 on bad arguments. */
int orc_trunc_order(double z, double tol)
{
    if (!(tol > 0.0) || !(z >= 0.0) || !isfinite(z)) return -1;
    int kmax = (int)ceil(z) + 64;
    for (;;) {
        double *J = (double *)malloc(sizeof(double) * ((size_t)kmax + 1));
        if (!J) return -1;
        orc_bessel_j(z, kmax, J);
        int found = -1;
        for (int k = 1; k <= kmax; ++k) {
            if ((double)k > z && fabs(J[k]) < tol) { found = k; break; }
        }
        free(J);
        if (found >= 0) return found - 1;
        kmax *= 2;
    }
}

/* Spectral shift and scale (Sect. 2.2): b = (Emax+Emin)/2,
 * eps = alpha (Emax-Emin), a = (Emax-Emin+eps)/2. */
int orc_scale(double emin, double emax, double alpha, double *a, double *b)
{
    if (!(emax > emin) || !(alpha >= 0.0)) return -1;
    double eps = alpha * (emax - emin);
    *b = 0.5 * (emax + emin);
    *a = 0.5 * (emax - emin + eps);
    return 0;
}

/* Expansion weights of eq. (U_1) with the prefactor and the factor 2 folded
 * in: gamma_0 = e^{-i b dt} c_0, gamma_k = 2 e^{-i b dt} c_k (k >= 1), with
 * c_k = (-i)^k J_k(a dt).  gamma is complex[M+1] (interleaved re, im). */
int orc_coeffs(double a, double b, double dt, int M, double *gamma)
{
    if (M < 0 || !gamma) return -1;
    double *J = (double *)malloc(sizeof(double) * ((size_t)M + 1));
    if (!J) return -1;
    orc_bessel_j(a * dt, M, J);
    cplx phase = cos(b * dt) - I * sin(b * dt);
    for (int k = 0; k <= M; ++k) {
        cplx mi; /* (-i)^k */
        switch (k % 4) {
        case 0: mi = 1.0; break;
        case 1: mi = -I; break;
        case 2: mi = -1.0; break;
        default: mi = I; break;
        }
        cplx g = phase * mi * J[k];
        if (k > 0) g *= 2.0;
        gamma[2 * k] = creal(g);
        gamma[2 * k + 1] = cimag(g);
    }
    free(J);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sparse matrices.  All Hamiltonians here are explicit CSR with complex     */
/* values (interleaved re, im), rows sorted by column.                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n, nnz;
    int64_t *rowptr;
    int64_t *col;
    double *val; /* complex[nnz] */
} orc_csr;

static void csr_free(orc_csr *m)
{
    free(m->rowptr); free(m->col); free(m->val);
    memset(m, 0, sizeof(*m));
}

/* Growable triplet list used by the builders. */
typedef struct { int64_t r, c; double re, im; } trip;
typedef struct { trip *t; int64_t n, cap; } triplist;

static int tl_push(triplist *l, int64_t r, int64_t c, double re, double im)
{
    if (l->n == l->cap) {
        int64_t nc = l->cap ? 2 * l->cap : 1024;
        trip *nt = (trip *)realloc(l->t, sizeof(trip) * (size_t)nc);
        if (!nt) return -1;
        l->t = nt; l->cap = nc;
    }
    l->t[l->n].r = r; l->t[l->n].c = c; l->t[l->n].re = re; l->t[l->n].im = im;
    l->n++;
    return 0;
}

static int trip_cmp(const void *x, const void *y)
{
    const trip *a = (const trip *)x, *b = (const trip *)y;
    if (a->r != b->r) return a->r < b->r ? -1 : 1;
    if (a->c != b->c) return a->c < b->c ? -1 : 1;
    return 0;
}

/* Sort triplets, merge duplicates by summation, emit CSR. */
static int tl_to_csr(triplist *l, int64_t n, orc_csr *m)
{
    qsort(l->t, (size_t)l->n, sizeof(trip), trip_cmp);
    int64_t w = 0;
    for (int64_t i = 0; i < l->n; ++i) {
        if (w > 0 && l->t[w - 1].r == l->t[i].r && l->t[w - 1].c == l->t[i].c) {
            l->t[w - 1].re += l->t[i].re;
            l->t[w - 1].im += l->t[i].im;
        } else {
            l->t[w++] = l->t[i];
        }
    }
    m->n = n; m->nnz = w;
    m->rowptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    m->col = (int64_t *)malloc(sizeof(int64_t) * (size_t)(w ? w : 1));
    m->val = (double *)malloc(sizeof(double) * 2 * (size_t)(w ? w : 1));
    if (!m->rowptr || !m->col || !m->val) { csr_free(m); return -1; }
    for (int64_t i = 0; i < w; ++i) {
        m->rowptr[l->t[i].r + 1]++;
        m->col[i] = l->t[i].c;
        m->val[2 * i] = l->t[i].re;
        m->val[2 * i + 1] = l->t[i].im;
    }
    for (int64_t r = 0; r < n; ++r) m->rowptr[r + 1] += m->rowptr[r];
    return 0;
}

/* Handle table so Python can keep matrices alive between calls. */
#define ORC_MAXH 64
static orc_csr g_mats[ORC_MAXH];
static int g_used[ORC_MAXH];

static int store_matrix(orc_csr *m)
{
    for (int h = 0; h < ORC_MAXH; ++h) {
        if (!g_used[h]) { g_mats[h] = *m; g_used[h] = 1; return h; }
    }
    csr_free(m);
    return -1;
}

static orc_csr *get_matrix(int h)
{
    if (h < 0 || h >= ORC_MAXH || !g_used[h]) return NULL;
    return &g_mats[h];
}

void orc_free_matrix(int h)
{
    orc_csr *m = get_matrix(h);
    if (m) { csr_free(m); g_used[h] = 0; }
}

int64_t orc_matrix_nnz(int h) { orc_csr *m = get_matrix(h); return m ? m->nnz : -1; }
int64_t orc_matrix_n(int h) { orc_csr *m = get_matrix(h); return m ? m->n : -1; }

/* Copy a stored matrix out (rowptr int64[n+1], col int64[nnz], val c128[nnz]). */
int orc_matrix_export(int h, int64_t *rowptr, int64_t *col, double *val)
{
    orc_csr *m = get_matrix(h);
    if (!m) return -1;
    memcpy(rowptr, m->rowptr, sizeof(int64_t) * ((size_t)m->n + 1));
    memcpy(col, m->col, sizeof(int64_t) * (size_t)m->nnz);
    memcpy(val, m->val, sizeof(double) * 2 * (size_t)m->nnz);
    return 0;
}

/* Import an arbitrary CSR (e.g. a test matrix). */
int orc_matrix_import(int64_t n, int64_t nnz, const int64_t *rowptr,
                      const int64_t *col, const double *val)
{
    orc_csr m;
    m.n = n; m.nnz = nnz;
    m.rowptr = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    m.col = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz ? nnz : 1));
    m.val = (double *)malloc(sizeof(double) * 2 * (size_t)(nnz ? nnz : 1));
    if (!m.rowptr || !m.col || !m.val) { csr_free(&m); return -1; }
    memcpy(m.rowptr, rowptr, sizeof(int64_t) * ((size_t)n + 1));
    memcpy(m.col, col, sizeof(int64_t) * (size_t)nnz);
    memcpy(m.val, val, sizeof(double) * 2 * (size_t)nnz);
    return store_matrix(&m);
}

/* 1D finite-difference Hamiltonian (Sect. 3.1): H = -1/2 d^2/dx^2 + V(x) on
 * n equally spaced points with spacing dx (m = hbar = 1), three-point
 * Laplacian, Dirichlet ends (the stencil is truncated at both ends). */
int orc_build_chain1d(int64_t n, double dx, const double *V)
{
    if (n < 1 || !(dx > 0.0) || !V) return -1;
    triplist l = {0};
    double hop = -0.5 / (dx * dx);
    for (int64_t j = 0; j < n; ++j) {
        if (j > 0) tl_push(&l, j, j - 1, hop, 0.0);
        tl_push(&l, j, j, 1.0 / (dx * dx) + V[j], 0.0);
        if (j + 1 < n) tl_push(&l, j, j + 1, hop, 0.0);
    }
    orc_csr m;
    int rc = tl_to_csr(&l, n, &m);
    free(l.t);
    if (rc) return -1;
    return store_matrix(&m);
}

/* Honeycomb-lattice ribbon, eq. (model): H = -t sum_<ij> (c_i^+ c_j + h.c.)
 * + sum_j eps_j n_j, drawn as a brick wall on a W x L grid, site index
 * y*L + x.  edge = 0 (zigzag ribbon): every site bonds to (x+-1, y), plus
 * (x, y+1) when x+y is even or (x, y-1) when x+y is odd.  edge = 1
 * (armchair ribbon): every site bonds to (x, y+-1), plus (x+1, y) when x+y
 * is even or (x-1, y) when odd.  Open boundaries. */
int orc_build_honeycomb(int64_t W, int64_t L, int edge, double t, const double *eps)
{
    if (W < 1 || L < 1 || (edge != 0 && edge != 1) || !eps) return -1;
    triplist l = {0};
    for (int64_t y = 0; y < W; ++y) {
        for (int64_t x = 0; x < L; ++x) {
            int64_t i = y * L + x;
            tl_push(&l, i, i, eps[i], 0.0);
            /* enumerate the candidate neighbours; keep those on the grid */
            int64_t nb[3][2];
            int cnt = 0;
            int even = ((x + y) % 2) == 0;
            if (edge == 0) {
                nb[cnt][0] = x - 1; nb[cnt][1] = y; cnt++;
                nb[cnt][0] = x + 1; nb[cnt][1] = y; cnt++;
                nb[cnt][0] = x; nb[cnt][1] = even ? y + 1 : y - 1; cnt++;
            } else {
                nb[cnt][0] = x; nb[cnt][1] = y - 1; cnt++;
                nb[cnt][0] = x; nb[cnt][1] = y + 1; cnt++;
                nb[cnt][0] = even ? x + 1 : x - 1; nb[cnt][1] = y; cnt++;
            }
            for (int q = 0; q < cnt; ++q) {
                int64_t xx = nb[q][0], yy = nb[q][1];
                if (xx < 0 || xx >= L || yy < 0 || yy >= W) continue;
                tl_push(&l, i, yy * L + xx, -t, 0.0);
            }
        }
    }
    orc_csr m;
    int rc = tl_to_csr(&l, W * L, &m);
    free(l.t);
    if (rc) return -1;
    return store_matrix(&m);
}

/* ------------------------------------------------------------------------ */
/* Holstein polaron basis, eq. (ghm): one spinless electron on L sites times */
/* phonon Fock states with total phonon number <= nph (the truncation of     */
/* Sect. 3.3).  Phonon configurations are ordered by total phonon number,    */
/* then lexicographically ascending in (n_1, ..., n_L) with n_1 most         */
/* significant.  State index = electron site * nconf + rank(phonon config):  */
/* the configurations of one electron site are contiguous.                  */
/* The oracle enumerates the configurations explicitly and looks them up by  */
/* binary search over an encoded key.                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int L, nph;
    int64_t count;
    uint8_t *occ;      /* occ[r*L + j] */
    uint64_t *keys;    /* sorted keys */
    int64_t *key_rank; /* rank for keys[i] */
} orc_basis;

static uint64_t occ_key(const uint8_t *n, int L, int nph)
{
    uint64_t k = 0;
    for (int j = 0; j < L; ++j) k = k * (uint64_t)(nph + 1) + n[j];
    return k;
}

static void gen_configs(orc_basis *B, uint8_t *cur, int pos, int remaining)
{
    if (pos == B->L - 1) {
        cur[pos] = (uint8_t)remaining;
        memcpy(B->occ + B->count * B->L, cur, (size_t)B->L);
        B->count++;
        return;
    }
    for (int v = 0; v <= remaining; ++v) {
        cur[pos] = (uint8_t)v;
        gen_configs(B, cur, pos + 1, remaining - v);
    }
}

static double binom(int n, int k)
{
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

static orc_basis *g_keysort_basis;
static int key_cmp(const void *x, const void *y)
{
    int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    uint64_t ka = occ_key(g_keysort_basis->occ + a * g_keysort_basis->L, g_keysort_basis->L, g_keysort_basis->nph);
    uint64_t kb = occ_key(g_keysort_basis->occ + b * g_keysort_basis->L, g_keysort_basis->L, g_keysort_basis->nph);
    return ka < kb ? -1 : (ka > kb ? 1 : 0);
}

static int basis_build(orc_basis *B, int L, int nph)
{
    memset(B, 0, sizeof(*B));
    /* keys must fit in 64 bits */
    if (L < 1 || nph < 0 || nph > 255 || L * log2((double)nph + 1.0) > 63.0) return -1;
    double cnt = binom(L + nph, nph);
    if (cnt > 5e7) return -1;
    B->L = L; B->nph = nph;
    B->occ = (uint8_t *)malloc((size_t)cnt * (size_t)L);
    uint8_t *cur = (uint8_t *)calloc((size_t)L, 1);
    if (!B->occ || !cur) { free(cur); return -1; }
    for (int T = 0; T <= nph; ++T) gen_configs(B, cur, 0, T);
    free(cur);
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)B->count);
    B->keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)B->count);
    B->key_rank = (int64_t *)malloc(sizeof(int64_t) * (size_t)B->count);
    if (!idx || !B->keys || !B->key_rank) { free(idx); return -1; }
    for (int64_t r = 0; r < B->count; ++r) idx[r] = r;
    g_keysort_basis = B;
    qsort(idx, (size_t)B->count, sizeof(int64_t), key_cmp);
    for (int64_t i = 0; i < B->count; ++i) {
        B->key_rank[i] = idx[i];
        B->keys[i] = occ_key(B->occ + idx[i] * L, L, nph);
    }
    free(idx);
    return 0;
}

static void basis_free(orc_basis *B)
{
    free(B->occ); free(B->keys); free(B->key_rank);
    memset(B, 0, sizeof(*B));
}

static int64_t basis_lookup(const orc_basis *B, const uint8_t *n)
{
    uint64_t k = occ_key(n, B->L, B->nph);
    int64_t lo = 0, hi = B->count - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (B->keys[mid] == k) return B->key_rank[mid];
        if (B->keys[mid] < k) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* Number of phonon configurations with total <= nph; the full dimension is
 * L times this (Sect. 3.3). */
int64_t orc_holstein_nconf(int L, int nph)
{
    return (int64_t)llround(binom(L + nph, nph));
}

/* Occupation table occ[r*L + j] (uint8) of the oracle's basis order. */
int orc_holstein_occupations(int L, int nph, uint8_t *occ)
{
    orc_basis B;
    if (basis_build(&B, L, nph)) return -1;
    memcpy(occ, B.occ, (size_t)B.count * (size_t)L);
    basis_free(&B);
    return 0;
}

/* Generalised Holstein Hamiltonian, eq. (ghm), spinless single electron:
 * H = sum_i Delta_i n_i - t sum_i (c_i^+ c_{i+1} + h.c.)
 *     - sum_i g_i w0 (b_i^+ + b_i) n_i + w0 sum_i b_i^+ b_i,
 * in the truncated basis above.  periodic != 0 closes the chain into a
 * ring (requires L >= 3); otherwise open ends.  g[i] is the dimensionless
 * coupling g_i of eq. (ghm). */
int orc_build_holstein(int L, int nph, double t, double w0, const double *g,
                       const double *Delta, int periodic)
{
    if (L < 1 || nph < 0 || !g || !Delta || (periodic && L < 3)) return -1;
    orc_basis B;
    if (basis_build(&B, L, nph)) return -1;
    triplist l = {0};
    uint8_t *nb = (uint8_t *)malloc((size_t)L);
    const int64_t C = B.count;  /* state (i, r) sits at i * C + r */
    for (int64_t r = 0; r < C; ++r) {
        const uint8_t *n = B.occ + r * L;
        int T = 0;
        for (int j = 0; j < L; ++j) T += n[j];
        for (int i = 0; i < L; ++i) {
            int64_t row = (int64_t)i * C + r;
            tl_push(&l, row, row, Delta[i] + w0 * T, 0.0);
            /* electron transfer to the neighbouring sites */
            int left = i - 1, right = i + 1;
            if (periodic) { left = (i - 1 + L) % L; right = (i + 1) % L; }
            if (left >= 0) tl_push(&l, row, (int64_t)left * C + r, -t, 0.0);
            if (right < L) tl_push(&l, row, (int64_t)right * C + r, -t, 0.0);
            /* column n + e_i: <n| b_i |n + e_i> = sqrt(n_i + 1) */
            if (T < nph) {
                memcpy(nb, n, (size_t)L); nb[i]++;
                int64_t rp = basis_lookup(&B, nb);
                double amp = -g[i] * w0 * sqrt((double)n[i] + 1.0);
                tl_push(&l, row, (int64_t)i * C + rp, amp, 0.0);
            }
            /* column n - e_i: <n| b_i^+ |n - e_i> = sqrt(n_i) */
            if (n[i] > 0) {
                memcpy(nb, n, (size_t)L); nb[i]--;
                int64_t rm = basis_lookup(&B, nb);
                double amp = -g[i] * w0 * sqrt((double)n[i]);
                tl_push(&l, row, (int64_t)i * C + rm, amp, 0.0);
            }
        }
    }
    free(nb);
    orc_csr m;
    int rc = tl_to_csr(&l, B.count * L, &m);
    free(l.t);
    basis_free(&B);
    if (rc) return -1;
    return store_matrix(&m);
}

/* ------------------------------------------------------------------------ */
/* Spectral bounds: Gershgorin discs (the paper does not state how Emin and  */
/* Emax are obtained; this is the reading used throughout).                  */
/* ------------------------------------------------------------------------ */
int orc_gershgorin(int h, double *emin, double *emax)
{
    orc_csr *m = get_matrix(h);
    if (!m || m->n < 1) return -1;
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = 0; i < m->n; ++i) {
        double d = 0.0, r = 0.0;
        for (int64_t p = m->rowptr[i]; p < m->rowptr[i + 1]; ++p) {
            cplx v = m->val[2 * p] + I * m->val[2 * p + 1];
            if (m->col[p] == i) d += creal(v);
            else r += cabs(v);
        }
        if (d - r < lo) lo = d - r;
        if (d + r > hi) hi = d + r;
    }
    *emin = lo; *emax = hi;
    return 0;
}

/* y = H x (plain CSR product). */
static void csr_apply(const orc_csr *m, const cplx *x, cplx *y)
{
    for (int64_t i = 0; i < m->n; ++i) {
        cplx s = 0.0;
        for (int64_t p = m->rowptr[i]; p < m->rowptr[i + 1]; ++p) {
            cplx v = m->val[2 * p] + I * m->val[2 * p + 1];
            s += v * x[m->col[p]];
        }
        y[i] = s;
    }
}

/* y = H~ x with H~ = (H - b)/a (Sect. 2.2). */
static void apply_scaled(const orc_csr *m, double a, double b, const cplx *x, cplx *y)
{
    csr_apply(m, x, y);
    for (int64_t i = 0; i < m->n; ++i) y[i] = (y[i] - b * x[i]) / a;
}

int orc_apply(int h, const double *x, double *y)
{
    orc_csr *m = get_matrix(h);
    if (!m) return -1;
    csr_apply(m, (const cplx *)x, (cplx *)y);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Chebyshev propagation (Sect. 2.2, eq. (U_1) and the recursion):           */
/*   v_0 = psi, v_1 = H~ v_0, v_{k+1} = 2 H~ v_k - v_{k-1},                  */
/*   psi(t+dt) = sum_{k=0}^{M} gamma_k v_k,                                  */
/* repeated K times with the same coefficients (computed once per dt).       */
/* norm_out[s] = <psi_s|psi_s> and energy_out[s] = <psi_s|H|psi_s> for the   */
/* state entering step s (either may be NULL).  psi is complex[n], in/out.   */
/* ------------------------------------------------------------------------ */
int orc_propagate(int h, double a, double b, int M, const double *gamma_ri,
                  double *psi_ri, int64_t K, double *norm_out, double *energy_out)
{
    orc_csr *m = get_matrix(h);
    if (!m || M < 0 || K < 0 || !(a > 0.0)) return -1;
    int64_t n = m->n;
    cplx *psi = (cplx *)psi_ri;
    const cplx *gamma = (const cplx *)gamma_ri;
    cplx *v0 = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *v1 = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *v2 = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *acc = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!v0 || !v1 || !v2 || !acc) { free(v0); free(v1); free(v2); free(acc); return -1; }
    for (int64_t s = 0; s < K; ++s) {
        memcpy(v0, psi, sizeof(cplx) * (size_t)n);
        apply_scaled(m, a, b, v0, v1);
        double nrm = 0.0, e = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            nrm += creal(conj(v0[i]) * v0[i]);
            e += creal(conj(v0[i]) * v1[i]);
        }
        if (norm_out) norm_out[s] = nrm;
        if (energy_out) energy_out[s] = a * e + b * nrm; /* <H> = a<H~> + b<1> */
        for (int64_t i = 0; i < n; ++i) {
            acc[i] = gamma[0] * v0[i];
            if (M >= 1) acc[i] += gamma[1] * v1[i];
        }
        for (int k = 1; k <= M - 1; ++k) {
            apply_scaled(m, a, b, v1, v2);
            for (int64_t i = 0; i < n; ++i) {
                v2[i] = 2.0 * v2[i] - v0[i];
                acc[i] += gamma[k + 1] * v2[i];
            }
            cplx *tmp = v0; v0 = v1; v1 = v2; v2 = tmp;
        }
        memcpy(psi, acc, sizeof(cplx) * (size_t)n);
    }
    free(v0); free(v1); free(v2); free(acc);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Reverse mode of the propagation above with respect to the diagonal of H.  */
/* L = sum_i mask_i |psi_K,i|^2 (a real objective of the final state);       */
/* gbar = dL/d conj(psi) convention: dL = Re sum conj(gbar_i) dpsi_i, so     */
/* gbar_K = 2 mask psi_K.  (a, b) and the weights gamma_k are held fixed.    */
/* For each step in reverse, with u_k the adjoint of v_k (u_{M+1} = 0):      */
/*   u_M = conj(gamma_M) gbar,                                               */
/*   u_k = conj(gamma_k) gbar + 2 H~ u_{k+1} - u_{k+2}      (1 <= k < M),    */
/*   u_0 = conj(gamma_0) gbar + H~ u_1 - u_2,                                */
/*   dL/dV_i += (1/a) Re[conj(u_1,i) v_0,i + 2 sum_{k=1}^{M-1}               */
/*                         conj(u_{k+1},i) v_k,i],                           */
/* and gbar of the preceding step is u_0.  H~ is real symmetric here, so it  */
/* is its own adjoint.  The forward states psi_s are kept for every step and */
/* each step's v_k are recomputed from psi_s before its reverse sweep.       */
/* mask is float64[n] (0/1 weights); dLdV float64[n] is overwritten;          */
/* gbar0_out (complex[n], may be NULL) receives the adjoint of psi_0.        */
/* psi_ri is the initial state (not modified).  L_out receives L.            */
/* ------------------------------------------------------------------------ */
int orc_adjoint(int h, double a, double b, int M, const double *gamma_ri,
                const double *psi0_ri, int64_t K, const double *mask,
                double *dLdV, double *gbar0_out, double *L_out)
{
    orc_csr *m = get_matrix(h);
    if (!m || M < 0 || K < 0 || !(a > 0.0)) return -1;
    int64_t n = m->n;
    const cplx *gamma = (const cplx *)gamma_ri;
    cplx *states = (cplx *)malloc(sizeof(cplx) * (size_t)n * (size_t)(K + 1));
    cplx *vk = (cplx *)malloc(sizeof(cplx) * (size_t)n * (size_t)(M + 2));
    cplx *uk = (cplx *)malloc(sizeof(cplx) * (size_t)n * (size_t)(M + 2));
    cplx *gbar = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!states || !vk || !uk || !gbar || !tmp) {
        free(states); free(vk); free(uk); free(gbar); free(tmp); return -1;
    }
    memcpy(states, psi0_ri, sizeof(cplx) * (size_t)n);
    for (int64_t s = 0; s < K; ++s) {
        memcpy(states + (s + 1) * n, states + s * n, sizeof(cplx) * (size_t)n);
        orc_propagate(h, a, b, M, gamma_ri, (double *)(states + (s + 1) * n), 1, NULL, NULL);
    }
    double L = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        cplx p = states[K * n + i];
        L += mask[i] * creal(conj(p) * p);
        gbar[i] = 2.0 * mask[i] * p;
        dLdV[i] = 0.0;
    }
    if (L_out) *L_out = L;
    for (int64_t s = K - 1; s >= 0; --s) {
        /* recompute v_0 .. v_M of step s */
        cplx *v = vk;
        memcpy(v, states + s * n, sizeof(cplx) * (size_t)n);
        if (M >= 1) apply_scaled(m, a, b, v, v + n);
        for (int k = 1; k <= M - 1; ++k) {
            apply_scaled(m, a, b, v + k * n, v + (k + 1) * n);
            for (int64_t i = 0; i < n; ++i)
                v[(k + 1) * n + i] = 2.0 * v[(k + 1) * n + i] - v[(k - 1) * n + i];
        }
        /* reverse sweep */
        cplx *u = uk;
        for (int64_t i = 0; i < n; ++i) u[(M + 1) * n + i] = 0.0;
        for (int64_t i = 0; i < n; ++i) u[M * n + i] = conj(gamma[M]) * gbar[i];
        for (int k = M - 1; k >= 0; --k) {
            apply_scaled(m, a, b, u + (k + 1) * n, tmp);
            double f = (k >= 1) ? 2.0 : 1.0;
            for (int64_t i = 0; i < n; ++i)
                u[k * n + i] = conj(gamma[k]) * gbar[i] + f * tmp[i] - u[(k + 2) * n + i];
        }
        for (int k = 0; k <= M - 1; ++k) {
            double f = (k >= 1) ? 2.0 : 1.0;
            for (int64_t i = 0; i < n; ++i)
                dLdV[i] += (f / a) * creal(conj(u[(k + 1) * n + i]) * v[k * n + i]);
        }
        memcpy(gbar, u, sizeof(cplx) * (size_t)n);
    }
    if (gbar0_out) memcpy(gbar0_out, gbar, sizeof(cplx) * (size_t)n);
    free(states); free(vk); free(uk); free(gbar); free(tmp);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Crank-Nicolson, eq. (CN): (1 + i H dt/2) psi_{s+1} = (1 - i H dt/2) psi_s */
/* for the tridiagonal 1D finite-difference H (same discretisation as        */
/* orc_build_chain1d), solved with the Thomas algorithm (Sect. 3.2).         */
/* ------------------------------------------------------------------------ */
int orc_crank_nicolson_1d(int64_t n, double dx, const double *V, double dt,
                          int64_t S, double *psi_ri)
{
    if (n < 2 || !(dx > 0.0) || S < 0) return -1;
    cplx *psi = (cplx *)psi_ri;
    double off = -0.5 / (dx * dx);
    cplx *rhs = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *cp = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *dp = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!rhs || !cp || !dp) { free(rhs); free(cp); free(dp); return -1; }
    cplx h = 0.5 * I * dt;
    for (int64_t s = 0; s < S; ++s) {
        /* right-hand side (1 - i H dt/2) psi */
        for (int64_t j = 0; j < n; ++j) {
            cplx Hp = (1.0 / (dx * dx) + V[j]) * psi[j];
            if (j > 0) Hp += off * psi[j - 1];
            if (j + 1 < n) Hp += off * psi[j + 1];
            rhs[j] = psi[j] - h * Hp;
        }
        /* Thomas algorithm on (1 + i H dt/2): sub = super = h*off,
         * diag_j = 1 + h*(1/dx^2 + V_j) */
        cplx sub = h * off, sup = h * off;
        cplx d0 = 1.0 + h * (1.0 / (dx * dx) + V[0]);
        cp[0] = sup / d0;
        dp[0] = rhs[0] / d0;
        for (int64_t j = 1; j < n; ++j) {
            cplx dj = 1.0 + h * (1.0 / (dx * dx) + V[j]);
            cplx den = dj - sub * cp[j - 1];
            cp[j] = (j + 1 < n) ? sup / den : 0.0;
            dp[j] = (rhs[j] - sub * dp[j - 1]) / den;
        }
        psi[n - 1] = dp[n - 1];
        for (int64_t j = n - 2; j >= 0; --j) psi[j] = dp[j] - cp[j] * psi[j + 1];
    }
    free(rhs); free(cp); free(dp);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Observables (Sect. 3.1 densities; Sect. 3.3 / Fig. 3 polaron quantities)  */
/* ------------------------------------------------------------------------ */
void orc_density(int64_t n, const double *psi_ri, double *rho)
{
    const cplx *psi = (const cplx *)psi_ri;
    for (int64_t i = 0; i < n; ++i) rho[i] = creal(conj(psi[i]) * psi[i]);
}

double orc_region_sum(int64_t n, const double *psi_ri, const uint8_t *mask)
{
    const cplx *psi = (const cplx *)psi_ri;
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (mask[i]) s += creal(conj(psi[i]) * psi[i]);
    return s;
}

/* Local electron density <n_i>, phonon number <b_i^+ b_i> and EP correlation
 * chi_ii = <n_i (b_i + b_i^+)> in the Holstein basis (Fig. 3). */
int orc_holstein_obs(int L, int nph, const double *psi_ri, double *n_i,
                     double *nph_i, double *chi_i)
{
    orc_basis B;
    if (basis_build(&B, L, nph)) return -1;
    const cplx *psi = (const cplx *)psi_ri;
    uint8_t *nb = (uint8_t *)malloc((size_t)L);
    for (int i = 0; i < L; ++i) { n_i[i] = 0.0; nph_i[i] = 0.0; chi_i[i] = 0.0; }
    const int64_t C = B.count;  /* state (i, r) sits at i * C + r */
    for (int64_t r = 0; r < C; ++r) {
        const uint8_t *n = B.occ + r * L;
        int T = 0;
        for (int j = 0; j < L; ++j) T += n[j];
        double w = 0.0; /* total weight of this phonon configuration */
        for (int i = 0; i < L; ++i) {
            cplx p = psi[(int64_t)i * C + r];
            double pp = creal(conj(p) * p);
            n_i[i] += pp;
            w += pp;
        }
        for (int j = 0; j < L; ++j) nph_i[j] += n[j] * w;
        for (int i = 0; i < L; ++i) {
            cplx p = psi[(int64_t)i * C + r];
            cplx bp = 0.0; /* ((b_i + b_i^+) psi)(i, r) */
            if (T < nph) {
                memcpy(nb, n, (size_t)L); nb[i]++;
                int64_t rp = basis_lookup(&B, nb);
                bp += sqrt((double)n[i] + 1.0) * psi[(int64_t)i * C + rp];
            }
            if (n[i] > 0) {
                memcpy(nb, n, (size_t)L); nb[i]--;
                int64_t rm = basis_lookup(&B, nb);
                bp += sqrt((double)n[i]) * psi[(int64_t)i * C + rm];
            }
            chi_i[i] += creal(conj(p) * bp);
        }
    }
    free(nb);
    basis_free(&B);
    return 0;
}
