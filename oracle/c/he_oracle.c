/*
 * Plain C build of the oracle's server evaluation (test infrastructure).
 *
 * The same steps as the numpy oracle (oracle/bfv.py server_conv / server_fc), written plainly in
 * C for timing on host cores: Alg. 1 / Alg. 2 server evaluation in the exact reading, with the
 * products in Z_q[X]/(X^N + 1) taken through a textbook transform (Sec. IV-A-1: the NTTs of the
 * masks rho and of the packed filters / weights are computed once at set-up and kept; each
 * evaluation transforms its inputs, multiplies coefficient-wise and transforms back).
 *
 *   transform   twisted cyclic form: coefficient i times psi^i, then an iterative radix-2
 *               decimation-in-time cyclic DFT with omega = psi^2 over natural order, so that
 *               output k is a(psi^(2k+1)); the inverse runs the DFT with omega^-1, then scales
 *               by N^-1 and psi^-i.  Every operation is a u64 product of two residues < 2^30
 *               reduced with %.
 *   conv        c0^(n) = sum_j c0_j rho_j^(n) - Delta sh_j fhat_j^(n); output poly n / g_o takes
 *               the residue class o_n of c0^(n), zero elsewhere; then + Delta sh' everywhere.
 *   fc          first n_o' coefficients of c0 rho_b - Delta sh w_b, + Delta ((d_b + sh'_b) mod t).
 *
 * Work is split over (limb, output channel) units with OpenMP when threads > 1.  Nothing here is
 * shared with the HIP library.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef uint64_t u64;

static u64 powmod(u64 a, u64 e, u64 q) {
    u64 r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = r * a % q;
        a = a * a % q;
        e >>= 1;
    }
    return r;
}

typedef struct {
    uint32_t N, logN;
    u64 q, ninv;
    u64 *twist, *untwist;   /* psi^i, psi^-i */
    u64 *wf, *wi;           /* stage powers: for length 2^m, entries [2^(m-1) - 1, 2^m - 1) hold w^j */
    uint32_t *rev;
} tables;

static int tables_make(tables *t, uint32_t N, u64 q, u64 psi) {
    memset(t, 0, sizeof(*t));
    t->N = N;
    t->q = q;
    while ((1u << t->logN) < N) ++t->logN;
    t->twist = malloc(N * sizeof(u64));
    t->untwist = malloc(N * sizeof(u64));
    t->wf = malloc(N * sizeof(u64));
    t->wi = malloc(N * sizeof(u64));
    t->rev = malloc(N * sizeof(uint32_t));
    if (!t->twist || !t->untwist || !t->wf || !t->wi || !t->rev) return -1;
    const u64 psi_inv = powmod(psi, q - 2, q);
    u64 p = 1, pi = 1;
    for (uint32_t i = 0; i < N; ++i) {
        t->twist[i] = p;
        t->untwist[i] = pi;
        p = p * psi % q;
        pi = pi * psi_inv % q;
        uint32_t r = 0;
        for (uint32_t b = 0; b < t->logN; ++b) r |= ((i >> b) & 1u) << (t->logN - 1 - b);
        t->rev[i] = r;
    }
    const u64 omega = psi * psi % q;
    for (uint32_t len = 2; len <= N; len <<= 1) {
        const u64 w = powmod(omega, N / len, q);
        const u64 winv = powmod(w, q - 2, q);
        u64 a = 1, b = 1;
        for (uint32_t j = 0; j < len / 2; ++j) {
            t->wf[len / 2 - 1 + j] = a;
            t->wi[len / 2 - 1 + j] = b;
            a = a * w % q;
            b = b * winv % q;
        }
    }
    t->ninv = powmod(N, q - 2, q);
    return 0;
}

static void tables_free(tables *t) {
    free(t->twist);
    free(t->untwist);
    free(t->wf);
    free(t->wi);
    free(t->rev);
}

/* In place: y = cyclic DFT of y (natural order in and out) with stage powers w. */
static void cyclic_dft(u64 *y, const tables *t, const u64 *w, u64 *tmp) {
    const uint32_t N = t->N;
    const u64 q = t->q;
    for (uint32_t i = 0; i < N; ++i) tmp[t->rev[i]] = y[i];
    memcpy(y, tmp, N * sizeof(u64));
    for (uint32_t len = 2; len <= N; len <<= 1) {
        const uint32_t half = len / 2;
        const u64 *wl = w + half - 1;
        for (uint32_t i = 0; i < N; i += len) {
            for (uint32_t j = 0; j < half; ++j) {
                const u64 u = y[i + j];
                const u64 v = y[i + j + half] * wl[j] % q;
                y[i + j] = (u + v) % q;
                y[i + j + half] = (u + q - v) % q;
            }
        }
    }
}

/* a (residues) -> its evaluations a(psi^(2k+1)) */
static void ntt(u64 *a, const tables *t, u64 *tmp) {
    for (uint32_t i = 0; i < t->N; ++i) a[i] = a[i] * t->twist[i] % t->q;
    cyclic_dft(a, t, t->wf, tmp);
}

static void intt(u64 *a, const tables *t, u64 *tmp) {
    cyclic_dft(a, t, t->wi, tmp);
    for (uint32_t i = 0; i < t->N; ++i) a[i] = a[i] * t->ninv % t->q * t->untwist[i] % t->q;
}

static u64 reduce_signed(int64_t a, u64 q) {
    int64_t r = a % (int64_t)q;
    return (u64)(r < 0 ? r + (int64_t)q : r);
}

static int set_threads(int threads) {
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
    return omp_get_max_threads();
#else
    (void)threads;
    return 1;
#endif
}

/*
 * Set-up: NTTs of signed integer rows for every limb.
 *   in   [rows][N] signed integers;  out [rows][L][N] evaluations mod q_l.
 */
int oracle_ntt_rows(uint32_t N, uint32_t L, const u64 *primes, const u64 *psis, uint32_t rows, const int64_t *in,
                    u64 *out, int threads) {
    tables *tb = calloc(L, sizeof(tables));
    if (!tb) return -1;
    int rc = 0;
    for (uint32_t l = 0; l < L; ++l)
        if (tables_make(&tb[l], N, primes[l], psis[l])) rc = -1;
    if (rc == 0) {
        set_threads(threads);
#pragma omp parallel for schedule(dynamic)
        for (int64_t u = 0; u < (int64_t)rows * L; ++u) {
            const uint32_t r = (uint32_t)(u / L), l = (uint32_t)(u % L);
            u64 *tmp = malloc(N * sizeof(u64));
            u64 *o = out + ((size_t)r * L + l) * N;
            for (uint32_t k = 0; k < N; ++k) o[k] = reduce_signed(in[(size_t)r * N + k], primes[l]);
            ntt(o, &tb[l], tmp);
            free(tmp);
        }
    }
    for (uint32_t l = 0; l < L; ++l) tables_free(&tb[l]);
    free(tb);
    return rc;
}

/*
 * Conv layer, server evaluation (Alg. 1).
 *   c0     [K_in][L][N] residues, coefficient form
 *   rho_h  [K_in][c_o][L][N]  NTT(rho_j^(n)) (oracle_ntt_rows)
 *   f_h    [K_in][c_o][L][N]  NTT(fhat_j^(n))
 *   sh     [K_in][N] in [0, t) or NULL;  sh_next [K_out][N] in [0, t) or NULL
 *   cls    [c_o] residue class o_n of each channel;  s slot stride;  g_o channels per output poly
 *   out    [K_out][L][N]
 */
int oracle_server_conv(uint32_t N, uint32_t L, const u64 *primes, const u64 *psis, const u64 *delta_l, uint32_t K_in,
                       uint32_t c_o, uint32_t g_o, uint32_t K_out, uint32_t s, const uint32_t *cls, const u64 *c0,
                       const u64 *rho_h, const u64 *f_h, const int64_t *sh, const int64_t *sh_next, u64 *out,
                       int threads) {
    tables *tb = calloc(L, sizeof(tables));
    u64 *X = malloc((size_t)K_in * L * N * sizeof(u64));   /* NTT(c0_j) per limb */
    u64 *S = malloc((size_t)K_in * L * N * sizeof(u64));   /* NTT(sh_j) per limb */
    if (!tb || !X || !S) return -1;
    int rc = 0;
    for (uint32_t l = 0; l < L; ++l)
        if (tables_make(&tb[l], N, primes[l], psis[l])) rc = -1;
    if (rc == 0) {
        set_threads(threads);
        memset(out, 0, (size_t)K_out * L * N * sizeof(u64));
#pragma omp parallel for schedule(dynamic)
        for (int64_t u = 0; u < (int64_t)K_in * L; ++u) {
            const uint32_t j = (uint32_t)(u / L), l = (uint32_t)(u % L);
            u64 *tmp = malloc(N * sizeof(u64));
            u64 *x = X + ((size_t)j * L + l) * N;
            memcpy(x, c0 + ((size_t)j * L + l) * N, N * sizeof(u64));
            ntt(x, &tb[l], tmp);
            if (sh) {
                u64 *y = S + ((size_t)j * L + l) * N;
                for (uint32_t k = 0; k < N; ++k) y[k] = reduce_signed(sh[(size_t)j * N + k], primes[l]);
                ntt(y, &tb[l], tmp);
            }
            free(tmp);
        }
#pragma omp parallel for schedule(dynamic)
        for (int64_t u = 0; u < (int64_t)L * c_o; ++u) {
            const uint32_t l = (uint32_t)(u / c_o), n = (uint32_t)(u % c_o);
            const u64 q = primes[l];
            u64 *A = calloc(N, sizeof(u64));
            u64 *P = calloc(N, sizeof(u64));
            u64 *tmp = malloc(N * sizeof(u64));
            for (uint32_t j = 0; j < K_in; ++j) {
                const u64 *x = X + ((size_t)j * L + l) * N;
                const u64 *r = rho_h + (((size_t)j * c_o + n) * L + l) * N;
                for (uint32_t k = 0; k < N; ++k) A[k] = (A[k] + x[k] * r[k] % q) % q;
                if (sh) {
                    const u64 *y = S + ((size_t)j * L + l) * N;
                    const u64 *f = f_h + (((size_t)j * c_o + n) * L + l) * N;
                    for (uint32_t k = 0; k < N; ++k) P[k] = (P[k] + y[k] * f[k] % q) % q;
                }
            }
            intt(A, &tb[l], tmp);
            if (sh) {
                intt(P, &tb[l], tmp);
                for (uint32_t k = 0; k < N; ++k) A[k] = (A[k] + q - P[k] * delta_l[l] % q) % q;
            }
            /* rotation-free extraction: residue class o_n of channel n into output poly n / g_o */
            u64 *o = out + ((size_t)(n / g_o) * L + l) * N;
            for (uint32_t k = cls[n]; k < N; k += s) o[k] = A[k];
            free(A);
            free(P);
            free(tmp);
        }
        if (sh_next) {
            for (uint32_t g = 0; g < K_out; ++g)
                for (uint32_t l = 0; l < L; ++l) {
                    const u64 q = primes[l];
                    u64 *o = out + ((size_t)g * L + l) * N;
                    for (uint32_t k = 0; k < N; ++k)
                        o[k] = (o[k] + reduce_signed(sh_next[(size_t)g * N + k], q) * delta_l[l] % q) % q;
                }
        }
    }
    for (uint32_t l = 0; l < L; ++l) tables_free(&tb[l]);
    free(tb);
    free(X);
    free(S);
    return rc;
}

/*
 * FC layer, server evaluation (Alg. 2).
 *   c0 [L][N]; rho_h, w_h [blocks][L][N] (NTTs of rho_b and w_b); sh [N] or NULL;
 *   d [blocks][n_o_p] signed bias; sh_next [blocks][n_o_p] or NULL; out [blocks][L][n_o_p].
 */
int oracle_server_fc(uint32_t N, uint32_t L, const u64 *primes, const u64 *psis, const u64 *delta_l, uint64_t t,
                     uint32_t blocks, uint32_t n_o_p, const u64 *c0, const u64 *rho_h, const u64 *w_h,
                     const int64_t *sh, const int64_t *d, const int64_t *sh_next, u64 *out, int threads) {
    tables *tb = calloc(L, sizeof(tables));
    u64 *X = malloc((size_t)L * N * sizeof(u64));
    u64 *S = malloc((size_t)L * N * sizeof(u64));
    if (!tb || !X || !S) return -1;
    int rc = 0;
    for (uint32_t l = 0; l < L; ++l)
        if (tables_make(&tb[l], N, primes[l], psis[l])) rc = -1;
    if (rc == 0) {
        set_threads(threads);
#pragma omp parallel for schedule(dynamic)
        for (int64_t l = 0; l < (int64_t)L; ++l) {
            u64 *tmp = malloc(N * sizeof(u64));
            memcpy(X + (size_t)l * N, c0 + (size_t)l * N, N * sizeof(u64));
            ntt(X + (size_t)l * N, &tb[l], tmp);
            if (sh) {
                for (uint32_t k = 0; k < N; ++k) S[(size_t)l * N + k] = reduce_signed(sh[k], primes[l]);
                ntt(S + (size_t)l * N, &tb[l], tmp);
            }
            free(tmp);
        }
#pragma omp parallel for schedule(dynamic)
        for (int64_t u = 0; u < (int64_t)L * blocks; ++u) {
            const uint32_t l = (uint32_t)(u / blocks), b = (uint32_t)(u % blocks);
            const u64 q = primes[l];
            u64 *A = malloc(N * sizeof(u64));
            u64 *P = malloc(N * sizeof(u64));
            u64 *tmp = malloc(N * sizeof(u64));
            const u64 *r = rho_h + ((size_t)b * L + l) * N;
            const u64 *w = w_h + ((size_t)b * L + l) * N;
            for (uint32_t k = 0; k < N; ++k) A[k] = X[(size_t)l * N + k] * r[k] % q;
            intt(A, &tb[l], tmp);
            if (sh) {
                for (uint32_t k = 0; k < N; ++k) P[k] = S[(size_t)l * N + k] * w[k] % q;
                intt(P, &tb[l], tmp);
                for (uint32_t k = 0; k < N; ++k) A[k] = (A[k] + q - P[k] * delta_l[l] % q) % q;
            }
            u64 *o = out + ((size_t)b * L + l) * n_o_p;
            for (uint32_t k = 0; k < n_o_p; ++k) {
                int64_t m = d[(size_t)b * n_o_p + k] + (sh_next ? sh_next[(size_t)b * n_o_p + k] : 0);
                m %= (int64_t)t;
                if (m < 0) m += (int64_t)t;
                o[k] = (A[k] + (u64)m * delta_l[l] % q) % q;
            }
            free(A);
            free(P);
            free(tmp);
        }
    }
    for (uint32_t l = 0; l < L; ++l) tables_free(&tb[l]);
    free(tb);
    free(X);
    free(S);
    return rc;
}

/* Threads an OpenMP region uses when asked for `threads` (0: the default). */
int oracle_threads(int threads) { return set_threads(threads); }
