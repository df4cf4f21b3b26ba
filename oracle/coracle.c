/*
 * Plain C oracle for the truncated FFT hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py may
 * load this library.  It shares no code with the HIP path.
 *
 * Definitions followed:
 *   co_fermat_dft_sampled  eq. (1) of Sect. 2 in R = Z/(2^N+1), theta = 2:
 *                          a_hat_j = zeta^(j') sum_{i<z} omega_L^(i j') a_i, at listed j.
 *   co_nega_dft_sampled    eq. (1) in R = (Z/mZ)[y]/(y^K+1), theta = y (Sect. 5.2).
 *   co_prime_dft_sampled   eq. (1) in R = Z/pZ, theta of order ord (Sect. 6): the
 *                          sum by Horner's rule at x = omega_L^(j'), times zeta^(j').
 *   co_zx_coeffs           u_k = sum_i g_i h_{k-i} over Z (schoolbook, Sect. 5.1).
 *   co_zmx_coeffs          u_k = sum_i g_i h_{k-i} mod m (schoolbook, Sect. 5.2).
 *   co_fingerprint         sum_k c_k r^k mod P (for Schwartz-Zippel checks).
 *
 * Residues mod 2^N+1 are W = N/32 little-endian 32-bit limbs plus a top word,
 * canonical in [0, 2^N].  Reduction mod 2^N+1 uses only 2^N = -1: an integer
 * is the alternating sum of its N-bit chunks.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ */
/* multi-limb helpers (32-bit limbs)                                   */
/* ------------------------------------------------------------------ */

/* r += a (n limbs each); returns carry out */
static uint32_t mp_add(uint32_t *r, const uint32_t *a, int n) {
    uint64_t c = 0;
    for (int i = 0; i < n; i++) {
        c += (uint64_t)r[i] + a[i];
        r[i] = (uint32_t)c;
        c >>= 32;
    }
    return (uint32_t)c;
}

/* r -= a (n limbs each); returns borrow out */
static uint32_t mp_sub(uint32_t *r, const uint32_t *a, int n) {
    int64_t b = 0;
    for (int i = 0; i < n; i++) {
        int64_t t = (int64_t)r[i] - a[i] + b;
        r[i] = (uint32_t)t;
        b = t >> 32; /* 0 or -1 */
    }
    return (uint32_t)(-b);
}

/* compare a and b (n limbs): -1, 0, +1 */
static int mp_cmp(const uint32_t *a, const uint32_t *b, int n) {
    for (int i = n - 1; i >= 0; i--) {
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Z/(2^N+1): reduction of a non-negative integer by chunk alternation  */
/* ------------------------------------------------------------------ */

/* out (W+1 limbs, canonical) = big mod 2^N+1, big has nb limbs.
 * big = sum_c chunk_c 2^(cN), 2^N = -1, so big = sum_c (-1)^c chunk_c. */
static void fm_reduce(uint32_t *out, const uint32_t *big, int nb, int W) {
    int A = W + 2; /* room for the sum of a few chunks */
    uint32_t *pos = calloc(A, 4), *neg = calloc(A, 4), *p = calloc(A, 4), *chunk = calloc(A, 4);
    p[0] = 1;
    p[W] = 1; /* p = 2^N + 1 */
    for (int c = 0; c * W < nb; c++) {
        memset(chunk, 0, 4 * A);
        for (int i = 0; i < W && c * W + i < nb; i++) chunk[i] = big[c * W + i];
        mp_add((c & 1) ? neg : pos, chunk, A);
    }
    /* reduce both sums below p */
    while (mp_cmp(pos, p, A) >= 0) mp_sub(pos, p, A);
    while (mp_cmp(neg, p, A) >= 0) mp_sub(neg, p, A);
    if (mp_cmp(pos, neg, A) >= 0) {
        mp_sub(pos, neg, A);
    } else {
        /* pos - neg + p */
        mp_add(pos, p, A);
        mp_sub(pos, neg, A);
    }
    memcpy(out, pos, 4 * (W + 1));
    free(pos);
    free(neg);
    free(p);
    free(chunk);
}

/* out = x * 2^e mod 2^N+1 for canonical x (W+1 limbs) */
static void fm_mul2exp(uint32_t *out, const uint32_t *x, uint64_t e, int W, uint32_t *scratch) {
    uint64_t twoN = 64ull * W;
    e %= twoN;
    int q = (int)(e >> 5), r = (int)(e & 31);
    int nb = W + 1 + q + 2;
    memset(scratch, 0, 4 * nb);
    for (int i = 0; i <= W; i++) {
        uint64_t v = (uint64_t)x[i] << r;
        scratch[i + q] |= (uint32_t)v;
        scratch[i + q + 1] |= (uint32_t)(v >> 32);
    }
    fm_reduce(out, scratch, nb, W);
}

typedef struct {
    int W;
    uint32_t L, l;
    uint64_t s, z;
    const uint32_t *a_limbs, *a_tops;
    const uint64_t *js;
    uint32_t *out_limbs, *out_tops;
    uint64_t j0, j1;
} fdft_job;

static uint32_t bitrev32(uint32_t j, uint32_t l) {
    uint32_t r = 0;
    for (uint32_t b = 0; b < l; b++) {
        r = (r << 1) | (j & 1);
        j >>= 1;
    }
    return r;
}

static void *fdft_worker(void *arg) {
    fdft_job *J = arg;
    int W = J->W;
    uint64_t twoN = 64ull * W;
    uint64_t w = twoN / J->L; /* omega_L = 2^w */
    int A = W + 3;
    uint32_t *x = calloc(W + 1, 4), *t = calloc(W + 1, 4), *acc = calloc(A, 4);
    uint32_t *scratch = calloc(3 * W + 8, 4), *res = calloc(W + 1, 4);
    uint32_t *tmp = calloc(A, 4);
    for (uint64_t jj = J->j0; jj < J->j1; jj++) {
        uint32_t jr = bitrev32((uint32_t)J->js[jj], J->l);
        memset(acc, 0, 4 * A);
        for (uint64_t i = 0; i < J->z; i++) {
            memcpy(x, J->a_limbs + i * W, 4 * W);
            x[W] = J->a_tops[i];
            /* exponent (w i j') mod 2N */
            uint64_t e = (uint64_t)(((u128)w * i * jr) % twoN);
            fm_mul2exp(t, x, e, W, scratch);
            memset(tmp, 0, 4 * A);
            memcpy(tmp, t, 4 * (W + 1));
            mp_add(acc, tmp, A);
        }
        fm_reduce(res, acc, A, W);
        uint64_t ez = (uint64_t)(((u128)(J->s % twoN) * jr) % twoN);
        fm_mul2exp(t, res, ez, W, scratch);
        memcpy(J->out_limbs + jj * W, t, 4 * W);
        J->out_tops[jj] = t[W];
    }
    free(x);
    free(t);
    free(acc);
    free(scratch);
    free(res);
    free(tmp);
    return NULL;
}

static void run_threads(void *jobs, size_t job_size, int nthreads, void *(*fn)(void *)) {
    pthread_t *th = calloc(nthreads, sizeof(pthread_t));
    for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, fn, (char *)jobs + t * job_size);
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    free(th);
}

/* Eq. (1) in Z/(2^N+1) at the listed output indices js. a has z canonical cells. */
int co_fermat_dft_sampled(uint32_t N, uint32_t L, uint64_t s, uint64_t z, const uint32_t *a_limbs,
                          const uint32_t *a_tops, uint64_t nj, const uint64_t *js, uint32_t *out_limbs,
                          uint32_t *out_tops, int nthreads) {
    if (N % 32 || L < 1 || (L & (L - 1)) || (2ull * N) % L) return 1;
    uint32_t l = 0;
    while ((1u << l) < L) l++;
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > nj) nthreads = nj ? (int)nj : 1;
    fdft_job *jobs = calloc(nthreads, sizeof(fdft_job));
    for (int t = 0; t < nthreads; t++) {
        fdft_job *J = &jobs[t];
        J->W = N / 32;
        J->L = L;
        J->l = l;
        J->s = s;
        J->z = z;
        J->a_limbs = a_limbs;
        J->a_tops = a_tops;
        J->js = js;
        J->out_limbs = out_limbs;
        J->out_tops = out_tops;
        J->j0 = nj * t / nthreads;
        J->j1 = nj * (t + 1) / nthreads;
    }
    run_threads(jobs, sizeof(fdft_job), nthreads, fdft_worker);
    free(jobs);
    return 0;
}

/* x * 2^e mod 2^N+1 for one canonical cell (exposed for pinning against Python ints). */
int co_fermat_mul2exp(uint32_t N, const uint32_t *x_limbs, uint32_t x_top, uint64_t e, uint32_t *out_limbs,
                      uint32_t *out_top) {
    int W = N / 32;
    uint32_t *x = calloc(W + 1, 4), *t = calloc(W + 1, 4), *scratch = calloc(3 * W + 8, 4);
    memcpy(x, x_limbs, 4 * W);
    x[W] = x_top;
    fm_mul2exp(t, x, e, W, scratch);
    memcpy(out_limbs, t, 4 * W);
    *out_top = t[W];
    free(x);
    free(t);
    free(scratch);
    return 0;
}

/* ------------------------------------------------------------------ */
/* (Z/mZ)[y]/(y^K+1)                                                   */
/* ------------------------------------------------------------------ */

typedef struct {
    uint32_t K, L, l;
    uint64_t m, s, z;
    const uint64_t *a;
    const uint64_t *js;
    uint64_t *out;
    uint64_t j0, j1;
} ndft_job;

/* acc += a * y^e (mod y^K+1, coefficients mod m) */
static void nega_addmul_theta(uint64_t *acc, const uint64_t *a, uint64_t e, uint32_t K, uint64_t m) {
    e %= 2ull * K;
    for (uint32_t i = 0; i < K; i++) {
        uint64_t pos = i + e; /* y^i y^e = y^(i+e) */
        uint64_t v = a[i];
        int neg = 0;
        while (pos >= K) {
            pos -= K;
            neg ^= 1;
        }
        if (neg && v) v = m - v;
        uint64_t t = acc[pos] + v;
        acc[pos] = t >= m ? t - m : t;
    }
}

static void *ndft_worker(void *arg) {
    ndft_job *J = arg;
    uint32_t K = J->K;
    uint64_t w = 2ull * K / J->L;
    uint64_t *acc = calloc(K, 8), *res = calloc(K, 8);
    for (uint64_t jj = J->j0; jj < J->j1; jj++) {
        uint32_t jr = bitrev32((uint32_t)J->js[jj], J->l);
        memset(acc, 0, 8 * K);
        for (uint64_t i = 0; i < J->z; i++) nega_addmul_theta(acc, J->a + i * K, w * i * jr, K, J->m);
        memset(res, 0, 8 * K);
        nega_addmul_theta(res, acc, (J->s % (2ull * K)) * jr, K, J->m);
        memcpy(J->out + jj * K, res, 8 * K);
    }
    free(acc);
    free(res);
    return NULL;
}

int co_nega_dft_sampled(uint32_t K, uint64_t m, uint32_t L, uint64_t s, uint64_t z, const uint64_t *a,
                        uint64_t nj, const uint64_t *js, uint64_t *out, int nthreads) {
    if (L < 1 || (L & (L - 1)) || (2ull * K) % L || m < 3 || !(m & 1) || m >= (1ull << 62)) return 1;
    uint32_t l = 0;
    while ((1u << l) < L) l++;
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > nj) nthreads = nj ? (int)nj : 1;
    ndft_job *jobs = calloc(nthreads, sizeof(ndft_job));
    for (int t = 0; t < nthreads; t++) {
        ndft_job *J = &jobs[t];
        J->K = K;
        J->L = L;
        J->l = l;
        J->m = m;
        J->s = s;
        J->z = z;
        J->a = a;
        J->js = js;
        J->out = out;
        J->j0 = nj * t / nthreads;
        J->j1 = nj * (t + 1) / nthreads;
    }
    run_threads(jobs, sizeof(ndft_job), nthreads, ndft_worker);
    free(jobs);
    return 0;
}

/* ------------------------------------------------------------------ */
/* eq. (1) in Z/pZ                                                     */
/* ------------------------------------------------------------------ */

static uint64_t powmod(uint64_t b, uint64_t e, uint64_t p) {
    uint64_t r = 1 % p;
    b %= p;
    while (e) {
        if (e & 1) r = (uint64_t)((u128)r * b % p);
        b = (uint64_t)((u128)b * b % p);
        e >>= 1;
    }
    return r;
}

typedef struct {
    uint64_t p, theta, ord, s, z;
    uint32_t L, l;
    const uint32_t *a;
    const uint64_t *js;
    uint32_t *out;
    uint64_t j0, j1;
} pdft_job;

static void *pdft_worker(void *arg) {
    pdft_job *J = arg;
    for (uint64_t jj = J->j0; jj < J->j1; jj++) {
        const uint64_t jr = bitrev32((uint32_t)J->js[jj], J->l);
        const uint64_t x = powmod(J->theta, (J->ord / J->L) * jr % J->ord, J->p);
        uint64_t acc = 0;
        for (uint64_t i = J->z; i-- > 0;) acc = (uint64_t)(((u128)acc * x + J->a[i]) % J->p);
        const uint64_t zj = powmod(J->theta, (J->s % J->ord) * jr % J->ord, J->p);
        J->out[jj] = (uint32_t)((u128)acc * zj % J->p);
    }
    return NULL;
}

int co_prime_dft_sampled(uint64_t p, uint64_t theta, uint64_t ord, uint32_t L, uint64_t s, uint64_t z,
                         const uint32_t *a, uint64_t nj, const uint64_t *js, uint32_t *out, int nthreads) {
    if (L < 1 || (L & (L - 1)) || ord % L || p < 3 || p >= (1ull << 32)) return 1;
    uint32_t l = 0;
    while ((1u << l) < L) l++;
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > nj) nthreads = nj ? (int)nj : 1;
    pdft_job *jobs = calloc(nthreads, sizeof(pdft_job));
    for (int t = 0; t < nthreads; t++) {
        pdft_job *J = &jobs[t];
        J->p = p;
        J->theta = theta;
        J->ord = ord;
        J->s = s;
        J->z = z;
        J->L = L;
        J->l = l;
        J->a = a;
        J->js = js;
        J->out = out;
        J->j0 = nj * t / nthreads;
        J->j1 = nj * (t + 1) / nthreads;
    }
    run_threads(jobs, sizeof(pdft_job), nthreads, pdft_worker);
    free(jobs);
    return 0;
}

/* ------------------------------------------------------------------ */
/* schoolbook products                                                 */
/* ------------------------------------------------------------------ */

typedef struct {
    const uint32_t *g, *h;
    uint64_t lg, lh;
    uint32_t gw, hw, ow;
    const uint64_t *ks;
    uint32_t *out;
    uint64_t k0, k1;
    int overflow;
} zx_job;

static void *zx_worker(void *arg) {
    zx_job *J = arg;
    int A = J->gw + J->hw + 3;
    if (A < (int)J->ow) A = J->ow;
    uint32_t *acc = calloc(A, 4);
    for (uint64_t kk = J->k0; kk < J->k1; kk++) {
        uint64_t k = J->ks[kk];
        memset(acc, 0, 4 * A);
        uint64_t lo = k >= J->lh - 1 ? k - (J->lh - 1) : 0;
        uint64_t hi = k < J->lg - 1 ? k : J->lg - 1;
        for (uint64_t i = lo; i <= hi && k < J->lg + J->lh - 1; i++) {
            const uint32_t *a = J->g + i * J->gw, *b = J->h + (k - i) * J->hw;
            /* acc += a * b, schoolbook over limbs */
            for (uint32_t x = 0; x < J->gw; x++) {
                uint64_t c = 0, ax = a[x];
                if (!ax) continue;
                uint32_t y = 0;
                for (; y < J->hw; y++) {
                    c += acc[x + y] + ax * b[y];
                    acc[x + y] = (uint32_t)c;
                    c >>= 32;
                }
                for (uint32_t t = x + y; c && (int)t < A; t++) {
                    c += acc[t];
                    acc[t] = (uint32_t)c;
                    c >>= 32;
                }
            }
        }
        for (int t = J->ow; t < A; t++)
            if (acc[t]) J->overflow = 1;
        memcpy(J->out + kk * J->ow, acc, 4 * J->ow);
    }
    free(acc);
    return NULL;
}

/* Exact Z[x] product coefficients u_k for k in ks; g: lg x gw limbs, h: lh x hw limbs,
 * out: nk x ow limbs.  Returns 2 if some coefficient does not fit in ow limbs. */
int co_zx_coeffs(const uint32_t *g, uint64_t lg, uint32_t gw, const uint32_t *h, uint64_t lh, uint32_t hw,
                 const uint64_t *ks, uint64_t nk, uint32_t *out, uint32_t ow, int nthreads) {
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > nk) nthreads = nk ? (int)nk : 1;
    zx_job *jobs = calloc(nthreads, sizeof(zx_job));
    for (int t = 0; t < nthreads; t++) {
        zx_job *J = &jobs[t];
        J->g = g;
        J->h = h;
        J->lg = lg;
        J->lh = lh;
        J->gw = gw;
        J->hw = hw;
        J->ow = ow;
        J->ks = ks;
        J->out = out;
        J->k0 = nk * t / nthreads;
        J->k1 = nk * (t + 1) / nthreads;
    }
    run_threads(jobs, sizeof(zx_job), nthreads, zx_worker);
    int of = 0;
    for (int t = 0; t < nthreads; t++) of |= jobs[t].overflow;
    free(jobs);
    return of ? 2 : 0;
}

typedef struct {
    const uint64_t *g, *h;
    uint64_t lg, lh, m;
    const uint64_t *ks;
    uint64_t *out;
    uint64_t k0, k1;
} zmx_job;

static void *zmx_worker(void *arg) {
    zmx_job *J = arg;
    for (uint64_t kk = J->k0; kk < J->k1; kk++) {
        uint64_t k = J->ks[kk];
        uint64_t lo = k >= J->lh - 1 ? k - (J->lh - 1) : 0;
        uint64_t hi = k < J->lg - 1 ? k : J->lg - 1;
        uint64_t r = 0;
        u128 acc = 0;
        int cnt = 0;
        for (uint64_t i = lo; i <= hi; i++) {
            acc += (u128)J->g[i] * J->h[k - i]; /* each product < 2^124 */
            if (++cnt == 8) {                   /* 8 * 2^124 = 2^127 < 2^128 */
                r = (uint64_t)(((u128)r + acc % J->m) % J->m);
                acc = 0;
                cnt = 0;
            }
        }
        r = (uint64_t)(((u128)r + acc % J->m) % J->m);
        J->out[kk] = r;
    }
    return NULL;
}

/* (Z/mZ)[x] product coefficients u_k mod m for k in ks (inputs in [0, m), m < 2^62). */
int co_zmx_coeffs(const uint64_t *g, uint64_t lg, const uint64_t *h, uint64_t lh, uint64_t m, const uint64_t *ks,
                  uint64_t nk, uint64_t *out, int nthreads) {
    if (m < 2 || m >= (1ull << 62)) return 1;
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > nk) nthreads = nk ? (int)nk : 1;
    zmx_job *jobs = calloc(nthreads, sizeof(zmx_job));
    for (int t = 0; t < nthreads; t++) {
        zmx_job *J = &jobs[t];
        J->g = g;
        J->h = h;
        J->lg = lg;
        J->lh = lh;
        J->m = m;
        J->ks = ks;
        J->out = out;
        J->k0 = nk * t / nthreads;
        J->k1 = nk * (t + 1) / nthreads;
    }
    run_threads(jobs, sizeof(zmx_job), nthreads, zmx_worker);
    free(jobs);
    return 0;
}

/* sum_k c_k r^k mod P, c_k given as w little-endian 32-bit limbs each (P < 2^63). */
uint64_t co_fingerprint(const uint32_t *limbs, uint64_t count, uint32_t w, uint64_t P, uint64_t r) {
    uint64_t acc = 0;
    for (uint64_t k = count; k-- > 0;) {
        uint64_t v = 0;
        for (uint32_t t = w; t-- > 0;) v = (uint64_t)((((u128)v << 32) + limbs[k * w + t]) % P);
        acc = (uint64_t)(((u128)acc * r + v) % P);
    }
    return acc;
}

/* same for 64-bit words (already reduced or not) */
uint64_t co_fingerprint64(const uint64_t *vals, uint64_t count, uint64_t P, uint64_t r) {
    uint64_t acc = 0;
    for (uint64_t k = count; k-- > 0;) acc = (uint64_t)(((u128)acc * r + vals[k] % P) % P);
    return acc;
}
