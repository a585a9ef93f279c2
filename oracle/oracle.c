/*
 * Plain CPU oracle for batched Lottery BP with OSD fallback.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU decoder.
 * Only the test suite, the package smoke check and the benchmark's CPU
 * baseline may load it; the product path never links, loads or calls it, and
 * it shares no source, header, table or helper with the GPU path.
 *
 * It is written to be read against the paper, not to be fast: one shot at a
 * time, flooding schedule, every quantity recomputed from its definition.
 *
 *   Prior LLR, VN/CN/LLR updates, hard decision, syndrome and termination:
 *       Algorithm 1 (normalized min-sum BP) and its description in Sec. II-B.
 *   Lottery policy: Algorithm 3 and Sec. III-B; CN selector index floor(r*N)
 *       and the VN-selector tie order from Sec. IV-B ("Optimized Lottery
 *       Pipeline"); first lottery after skipping 6 iterations (Sec. III-B).
 *   OSD-0: Algorithm 2 (sort, permute, first rank(H) independent columns,
 *       solve, zero-pad, un-permute).
 *   OSD-CS(w): not defined by the paper (it names higher-order OSD only);
 *       the combination sweep of Roffe, White, Burton and Campbell, Phys. Rev.
 *       Research 2, 043423 (2020): OSD-0, then every weight-1 pattern on the
 *       non-basis columns, then every weight-2 pattern among the first w
 *       non-basis columns; the minimum-Hamming-weight candidate wins.
 *   Int3.4 fixed point: Sec. VII-A (quantization analysis).
 *   Random numbers: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel
 *       random numbers: as easy as 1, 2, 3", SC'11).
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - float messages are rounded to the storage format (fp32 or fp16, round to
 *     nearest even, saturating at the largest finite value) where they are
 *     stored (prior, V2C, C2V); arithmetic in between is fp64;
 *   - V2C in "message flip" mode is the extrinsic sum mu + sum_{c' != c} beta
 *     in ascending c'; in "LLR flip" mode it is lambda - beta;
 *   - sigma_i = fl32(1 - 2^-(i+1)); Int3.4: |beta| = mag - (mag >> (i+1)),
 *     constant k/8: (k*mag) >> 3;
 *   - sgn(0) = +1; a check of degree 1 sends magnitude CAP;
 *   - hard decision lambda <= tau, tau = 2^-12 for float, 0 for Int3.4;
 *   - the lottery runs at the end of iteration i for K <= i <= I-2 and flips
 *     the messages v* sends in the next check-node update ("message flip") or
 *     lambda_{v*} itself ("LLR flip");
 *   - VN selector key: most unsatisfied checks, then smallest
 *     floor(|lambda| * 2^12) (|lambda| for Int3.4), then smallest column;
 *   - r = (x >> 32) / 2^32 with x = Philox word 0 of counter
 *     (shot_id, i, 0, 0) and key (seed, 0); the selected check is the
 *     ((x >> 32) * N >> 32)-th unsatisfied check in ascending order;
 *   - OSD sorts (lambda, column) ascending, stable; lambda is that of the last
 *     BP iteration.
 */
#include <float.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_FP32 0
#define ORC_FP16 1
#define ORC_INT8 2
#define ORC_FP64 3

#define ORC_FLIP_MSG 0
#define ORC_FLIP_LLR 1

#define ORC_OSD_NONE 0
#define ORC_OSD_0 1
#define ORC_OSD_CS 2

#define ORC_FLAG_CONVERGED 1
#define ORC_FLAG_OSD 2
#define ORC_FLAG_OSD_INCONSISTENT 4

#define CAP_FLOAT 1024.0
#define TAU_FLOAT (1.0 / 4096.0)

typedef struct {
    int32_t max_iter;
    int32_t scale_mode; /* 0: sigma_i = 1 - 2^-(i+1); 1: constant */
    double scale;       /* constant scale */
    int32_t msg;        /* ORC_FP32 / ORC_FP16 / ORC_INT8 / ORC_FP64 */
    int32_t lottery;
    int32_t lottery_skip;
    int32_t flip;
    int32_t osd;
    int32_t osd_order;
    int32_t early_stop; /* 1 normally; 0 keeps iterating (test hook) */
    int32_t policy;     /* lottery design-space variant: CN rule in bits 0-1, VN rule in bits 4-5 */
    int32_t fx_int;     /* fixed point Int x.y (ORC_INT8): x integer bits ... */
    int32_t fx_frac;    /* ... and y fraction bits plus a sign bit; 0, 0 means Int3.4 */
    uint64_t seed;
} orc_params;

typedef struct {
    int m, n, nnz;
    const int32_t *rp, *ci; /* CSR (row pointers, column of each edge) */
    int32_t *cp, *cr, *ce;  /* CSC: column pointers, row and CSR edge id of each entry, ascending row */
} ocode;

/* ------------------------------------------------------------------ Philox */

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

/* Philox4x64 with 10 rounds: each round multiplies counter words 0 and 2 by the
 * two round constants, swaps and xors the halves with words 1, 3 and the key;
 * the key is bumped by the two Weyl constants between rounds. */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(0xD2E7470EE14C6C93ULL, x0, &hi0, &lo0);
        mulhilo64(0xCA5A826395121157ULL, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------- storage rounding */

static double rne_fp16(double x) {
    if (x == 0.0 || isnan(x)) return x;
    double a = fabs(x);
    int e;
    frexp(a, &e);          /* a = f * 2^e, f in [0.5, 1) */
    int q = e - 11;        /* 11 significant bits */
    if (q < -24) q = -24;  /* subnormal quantum */
    double r = ldexp(nearbyint(ldexp(a, -q)), q);
    if (r > 65504.0) r = 65504.0; /* saturate instead of overflowing to inf */
    return copysign(r, x);
}

static double rne_fp32(double x) {
    float f = (float)x;
    if (isinf(f)) f = copysignf(FLT_MAX, f);
    return (double)f;
}

double orc_store(int fmt, double x) {
    if (fmt == ORC_FP32) return rne_fp32(x);
    if (fmt == ORC_FP16) return rne_fp16(x);
    return x;
}

/* Fixed point Int x.y (Sec. VII-A, quantization study): a sign bit, x integer
 * and y fraction bits, i.e. integers in units of 2^-y saturated symmetrically
 * to +-(2^(x+y) - 1).  The prior is 2^y mu rounded to nearest even, then
 * saturated.  Int3.4 (8 bits, LSB 1/16, +-127) is the paper's choice. */
int orc_prior_fixed(double p, int x, int y) {
    const double qmax = (double)((1 << (x + y)) - 1);
    double mu = log((1.0 - p) / p);
    double q = nearbyint(ldexp(mu, y));
    if (q > qmax) q = qmax;
    if (q < -qmax) q = -qmax;
    return (int)q;
}

int orc_prior_int8(double p) { return orc_prior_fixed(p, 3, 4); }

static int fx_x(const orc_params *P) { return (P->fx_int | P->fx_frac) ? P->fx_int : 3; }
static int fx_y(const orc_params *P) { return (P->fx_int | P->fx_frac) ? P->fx_frac : 4; }

static int satq(long x, long qmax) { return x > qmax ? (int)qmax : (x < -qmax ? (int)-qmax : (int)x); }

static double sigma_float(const orc_params *P, int i) {
    if (P->scale_mode == 1) return (double)(float)P->scale;
    return (double)(float)(1.0 - ldexp(1.0, -(i + 1)));
}

static int scale_int8(const orc_params *P, int i, int mag) {
    if (P->scale_mode == 1) {
        int k = (int)lround(P->scale * 8.0);
        return (k * mag) >> 3;
    }
    int sh = i + 1 > 30 ? 30 : i + 1;
    return mag - (mag >> sh);
}

/* Words 0 and 1 of the Philox block of (shot, iteration): word 0 picks the
 * check, word 1 the neighbour when that choice is random too. */
static void lottery_draw(uint64_t seed, uint64_t shot_id, int i, uint64_t *w0, uint64_t *w1) {
    uint64_t ctr[4] = {shot_id, (uint64_t)i, 0, 0}, key[2] = {seed, 0}, out[4];
    orc_philox4x64_10(ctr, key, out);
    *w0 = out[0];
    *w1 = out[1];
}

/* ------------------------------------------------------------------ BP */

typedef struct {
    double *mu, *alpha, *beta, *lam;
    long *imu, *ialpha, *ibeta, *ilam;
    uint8_t *shat, *sprev;
    int *ulist;
} work;

/* Lottery (Algorithm 3) for iteration i.  U uses the previous iteration's
 * syndrome estimate.  Returns v* or -1 when U is empty.
 *
 * Design space of the selection (Sec. III-B, Table I), P->policy:
 *   CN rule (bits 0-1): 0 = a random check of U (Algorithm 3);
 *                       1 = worst check: the check of U with the most
 *                           neighbours in the current hard decision, the
 *                           smallest index among equals.
 *   VN rule (bits 4-5): 0 = the proposed key: most neighbouring checks in U,
 *                           then smallest Q(|lambda|), then smallest column
 *                           (Algorithm 3 and Sec. IV-B);
 *                       1 = the same two criteria in the other order
 *                           (smallest Q first, then most checks in U), as
 *                           Sec. III-B words the proposed policy;
 *                       2 = unreliable neighbour: smallest Q, then column;
 *                       3 = a random neighbour.
 * Random draws: r0 = (word 0 >> 32) / 2^32 picks the check, index
 * floor(r0 |U|); r1 = (word 1 >> 32) / 2^32 picks the neighbour among the
 * check's columns in ascending order. */
static int lottery_pick(const ocode *C, const orc_params *P, uint64_t shot_id, int i,
                        const uint8_t *s, const uint8_t *sprev, int *ulist,
                        const double *lamf, const long *lami, const uint8_t *ehat) {
    const int cn_rule = P->policy & 3, vn_rule = (P->policy >> 4) & 3;
    int N = 0;
    for (int c = 0; c < C->m; ++c)
        if (sprev[c] != s[c]) ulist[N++] = c;
    if (N == 0) return -1;
    uint64_t x0, x1;
    lottery_draw(P->seed, shot_id, i, &x0, &x1);
    int cstar;
    if (cn_rule == 1) {
        int best = -1;
        cstar = -1;
        for (int u = 0; u < N; ++u) {
            int c = ulist[u], cnt = 0;
            for (int e = C->rp[c]; e < C->rp[c + 1]; ++e) cnt += ehat[C->ci[e]];
            if (cnt > best) { best = cnt; cstar = c; }   /* ascending c: first maximum wins */
        }
    } else {
        uint64_t k = ((x0 >> 32) * (uint64_t)N) >> 32; /* floor(r * N) */
        cstar = ulist[k];
    }
    if (vn_rule == 3) {
        const int deg = C->rp[cstar + 1] - C->rp[cstar];
        uint64_t k = ((x1 >> 32) * (uint64_t)deg) >> 32;
        return C->ci[C->rp[cstar] + (int)k];
    }
    int best_v = -1, best_cnt = -1;
    long long best_q = 0;
    for (int e = C->rp[cstar]; e < C->rp[cstar + 1]; ++e) {
        int v = C->ci[e];
        int cnt = 0;
        for (int t = C->cp[v]; t < C->cp[v + 1]; ++t)
            if (sprev[C->cr[t]] != s[C->cr[t]]) ++cnt;
        long long q;
        if (lami) q = labs(lami[v]);
        else {
            double a = fabs(lamf[v]) * 4096.0;
            q = a >= 4.0e18 ? (long long)4.0e18 : (long long)floor(a);
        }
        int better;
        if (best_v < 0) better = 1;
        else if (vn_rule == 0) better = cnt > best_cnt || (cnt == best_cnt && (q < best_q || (q == best_q && v < best_v)));
        else if (vn_rule == 1) better = q < best_q || (q == best_q && (cnt > best_cnt || (cnt == best_cnt && v < best_v)));
        else better = q < best_q || (q == best_q && v < best_v);
        if (better) { best_v = v; best_cnt = cnt; best_q = q; }
    }
    return best_v;
}

/* One shot, float messages (fp32 / fp16 storage or pure fp64). */
static void bp_float(const ocode *C, const orc_params *P, const double *prior, uint64_t shot_id,
                     const uint8_t *s, uint8_t *ehat, int *iters, int *conv, double *lam_out, work *W) {
    const int m = C->m, n = C->n, fmt = P->msg, I = P->max_iter;
    double *mu = W->mu, *alpha = W->alpha, *beta = W->beta, *lam = W->lam;
    for (int v = 0; v < n; ++v) mu[v] = orc_store(fmt, log((1.0 - prior[v]) / prior[v])); /* Algorithm 1: prior LLR */
    for (int e = 0; e < C->nnz; ++e) beta[e] = 0.0;
    for (int v = 0; v < n; ++v) lam[v] = mu[v];
    int flip_v = -1;
    *conv = 0;
    *iters = I;
    for (int i = 0; i < I; ++i) {
        /* VN update (Algorithm 1) */
        for (int c = 0; c < m; ++c)
            for (int e = C->rp[c]; e < C->rp[c + 1]; ++e) {
                int v = C->ci[e];
                double a;
                if (i == 0) a = mu[v];
                else if (P->flip == ORC_FLIP_MSG) {
                    a = mu[v];
                    for (int t = C->cp[v]; t < C->cp[v + 1]; ++t)
                        if (C->cr[t] != c) a += beta[C->ce[t]];
                } else a = lam[v] - beta[e];
                if (P->flip == ORC_FLIP_MSG && v == flip_v) a = -a;
                alpha[e] = orc_store(fmt, a);
            }
        /* CN update (Algorithm 1) */
        double sig = sigma_float(P, i);
        for (int c = 0; c < m; ++c) {
            int deg = C->rp[c + 1] - C->rp[c];
            double m1 = INFINITY, m2 = INFINITY;
            int arg = -1, par = 0;
            for (int e = C->rp[c]; e < C->rp[c + 1]; ++e) {
                double x = fabs(alpha[e]);
                if (x < m1) { m2 = m1; m1 = x; arg = e; }
                else if (x < m2) m2 = x;
                par ^= (alpha[e] < 0.0);
            }
            if (deg == 1) m2 = CAP_FLOAT;
            for (int e = C->rp[c]; e < C->rp[c + 1]; ++e) {
                double mag = (e == arg) ? m2 : m1;
                int neg = s[c] ^ par ^ (alpha[e] < 0.0);
                double b = sig * mag;
                beta[e] = orc_store(fmt, neg ? -b : b);
            }
        }
        /* LLR update, hard decision, syndrome estimate (Algorithm 1) */
        for (int v = 0; v < n; ++v) {
            double l = mu[v];
            for (int t = C->cp[v]; t < C->cp[v + 1]; ++t) l += beta[C->ce[t]];
            lam[v] = l;
            ehat[v] = (l <= TAU_FLOAT);
        }
        int match = 1;
        for (int c = 0; c < m; ++c) {
            int x = 0;
            for (int e = C->rp[c]; e < C->rp[c + 1]; ++e) x ^= ehat[C->ci[e]];
            W->shat[c] = (uint8_t)x;
            if (x != s[c]) match = 0;
        }
        if (match && P->early_stop) { /* early termination (Algorithm 1) */
            *conv = 1;
            *iters = i + 1;
            break;
        }
        *conv = match;
        /* lottery (Algorithm 3) */
        flip_v = -1;
        if (P->lottery && i >= P->lottery_skip && i <= I - 2) {
            int vs = lottery_pick(C, P, shot_id, i, s, W->sprev, W->ulist, lam, NULL, ehat);
            if (vs >= 0) {
                if (P->flip == ORC_FLIP_MSG) flip_v = vs;
                else lam[vs] = -lam[vs];
            }
        }
        memcpy(W->sprev, W->shat, (size_t)m);
    }
    if (lam_out) memcpy(lam_out, lam, sizeof(double) * (size_t)n);
}

/* One shot, fixed-point messages (Int x.y, Int3.4 by default): exact integer arithmetic. */
static void bp_int8(const ocode *C, const orc_params *P, const double *prior, uint64_t shot_id,
                    const uint8_t *s, uint8_t *ehat, int *iters, int *conv, double *lam_out, work *W) {
    const int m = C->m, n = C->n, I = P->max_iter;
    long *mu = W->imu, *alpha = W->ialpha, *beta = W->ibeta, *lam = W->ilam;
    const int fx = fx_x(P), fy = fx_y(P);
    const long qmax = (1L << (fx + fy)) - 1;
    for (int v = 0; v < n; ++v) mu[v] = orc_prior_fixed(prior[v], fx, fy);
    for (int e = 0; e < C->nnz; ++e) beta[e] = 0;
    for (int v = 0; v < n; ++v) lam[v] = mu[v];
    int flip_v = -1;
    *conv = 0;
    *iters = I;
    for (int i = 0; i < I; ++i) {
        for (int c = 0; c < m; ++c)
            for (int e = C->rp[c]; e < C->rp[c + 1]; ++e) {
                int v = C->ci[e];
                long a;
                if (i == 0) a = mu[v];
                else if (P->flip == ORC_FLIP_MSG) {
                    a = mu[v];
                    for (int t = C->cp[v]; t < C->cp[v + 1]; ++t)
                        if (C->cr[t] != c) a += beta[C->ce[t]];
                } else a = lam[v] - beta[e];
                if (P->flip == ORC_FLIP_MSG && v == flip_v) a = -a;
                alpha[e] = satq(a, qmax);
            }
        for (int c = 0; c < m; ++c) {
            int deg = C->rp[c + 1] - C->rp[c];
            long m1 = 1L << 40, m2 = 1L << 40;
            int arg = -1, par = 0;
            for (int e = C->rp[c]; e < C->rp[c + 1]; ++e) {
                long x = labs(alpha[e]);
                if (x < m1) { m2 = m1; m1 = x; arg = e; }
                else if (x < m2) m2 = x;
                par ^= (alpha[e] < 0);
            }
            if (deg == 1) m2 = qmax;
            for (int e = C->rp[c]; e < C->rp[c + 1]; ++e) {
                int mag = (int)((e == arg) ? m2 : m1);
                int neg = s[c] ^ par ^ (alpha[e] < 0);
                int b = scale_int8(P, i, mag);
                beta[e] = neg ? -b : b;
            }
        }
        for (int v = 0; v < n; ++v) {
            long l = mu[v];
            for (int t = C->cp[v]; t < C->cp[v + 1]; ++t) l += beta[C->ce[t]];
            lam[v] = l;
            ehat[v] = (l <= 0);
        }
        int match = 1;
        for (int c = 0; c < m; ++c) {
            int x = 0;
            for (int e = C->rp[c]; e < C->rp[c + 1]; ++e) x ^= ehat[C->ci[e]];
            W->shat[c] = (uint8_t)x;
            if (x != s[c]) match = 0;
        }
        if (match && P->early_stop) {
            *conv = 1;
            *iters = i + 1;
            break;
        }
        *conv = match;
        flip_v = -1;
        if (P->lottery && i >= P->lottery_skip && i <= I - 2) {
            int vs = lottery_pick(C, P, shot_id, i, s, W->sprev, W->ulist, NULL, lam, ehat);
            if (vs >= 0) {
                if (P->flip == ORC_FLIP_MSG) flip_v = vs;
                else lam[vs] = -lam[vs];
            }
        }
        memcpy(W->sprev, W->shat, (size_t)m);
    }
    if (lam_out)
        for (int v = 0; v < n; ++v) lam_out[v] = (double)lam[v];
}

/* ------------------------------------------------------------------ OSD */

typedef struct {
    double l;
    int col;
} keycol;

static int cmp_keycol(const void *a, const void *b) {
    const keycol *x = (const keycol *)a, *y = (const keycol *)b;
    if (x->l < y->l) return -1;
    if (x->l > y->l) return 1;
    return (x->col > y->col) - (x->col < y->col);
}

static inline int getbit(const uint64_t *row, int j) { return (int)((row[j >> 6] >> (j & 63)) & 1u); }

/* OSD-0 (Algorithm 2) and OSD-CS(order).  Returns 0 with ehat set, or 1 when
 * s is not in the column space of H (ehat untouched). */
static int osd_shot(const ocode *C, int mode, int order, const double *lam, const uint8_t *s, uint8_t *ehat) {
    const int m = C->m, n = C->n, W = (n + 1 + 63) / 64;
    keycol *kc = (keycol *)malloc(sizeof(keycol) * (size_t)n);
    int *pos = (int *)malloc(sizeof(int) * (size_t)n);
    int *pi = (int *)malloc(sizeof(int) * (size_t)n);
    uint64_t *A = (uint64_t *)calloc((size_t)m * (size_t)W, sizeof(uint64_t));
    uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)W);
    int *pivcol = (int *)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    uint8_t *isbasis = (uint8_t *)calloc((size_t)n, 1);
    int *T = (int *)malloc(sizeof(int) * (size_t)n);
    uint8_t *eperm = (uint8_t *)calloc((size_t)n, 1);
    int ret = 0;

    /* sort lambda ascending (stable: ties by column index) */
    for (int v = 0; v < n; ++v) { kc[v].l = lam[v] == 0.0 ? 0.0 : lam[v]; kc[v].col = v; }
    qsort(kc, (size_t)n, sizeof(keycol), cmp_keycol);
    for (int j = 0; j < n; ++j) { pi[j] = kc[j].col; pos[kc[j].col] = j; }
    /* permuted columns, augmented with s in column n */
    for (int c = 0; c < m; ++c) {
        uint64_t *row = A + (size_t)c * W;
        for (int e = C->rp[c]; e < C->rp[c + 1]; ++e) {
            int j = pos[C->ci[e]];
            row[j >> 6] |= 1ULL << (j & 63);
        }
        if (s[c]) row[n >> 6] |= 1ULL << (n & 63);
    }
    /* Gauss-Jordan elimination in permuted column order; the pivots are
     * the first rank(H) independent columns */
    int rank = 0;
    for (int j = 0; j < n && rank < m; ++j) {
        int r = -1;
        for (int q = rank; q < m; ++q)
            if (getbit(A + (size_t)q * W, j)) { r = q; break; }
        if (r < 0) continue;
        if (r != rank) {
            memcpy(tmp, A + (size_t)r * W, sizeof(uint64_t) * (size_t)W);
            memcpy(A + (size_t)r * W, A + (size_t)rank * W, sizeof(uint64_t) * (size_t)W);
            memcpy(A + (size_t)rank * W, tmp, sizeof(uint64_t) * (size_t)W);
        }
        const uint64_t *pr = A + (size_t)rank * W;
        for (int q = 0; q < m; ++q) {
            if (q == rank) continue;
            uint64_t *row = A + (size_t)q * W;
            if (getbit(row, j))
                for (int w = 0; w < W; ++w) row[w] ^= pr[w];
        }
        pivcol[rank] = j;
        isbasis[j] = 1;
        ++rank;
    }
    for (int q = rank; q < m; ++q)
        if (getbit(A + (size_t)q * W, n)) { ret = 1; goto done; }

    {
        int nt = 0;
        for (int j = 0; j < n; ++j)
            if (!isbasis[j]) T[nt++] = j;
        /* candidate t (at most two non-basis columns): e_S = s' + R t */
        int best_a = -1, best_b = -1;
        long best_cost = 0;
        for (int k = 0; k < rank; ++k) best_cost += getbit(A + (size_t)k * W, n);
        if (mode == ORC_OSD_CS) {
            for (int a = 0; a < nt; ++a) {
                long cost = 1;
                for (int k = 0; k < rank; ++k) {
                    const uint64_t *row = A + (size_t)k * W;
                    cost += getbit(row, n) ^ getbit(row, T[a]);
                }
                if (cost < best_cost) { best_cost = cost; best_a = a; best_b = -1; }
            }
            int w = order < nt ? order : nt;
            for (int a = 0; a < w; ++a)
                for (int b = a + 1; b < w; ++b) {
                    long cost = 2;
                    for (int k = 0; k < rank; ++k) {
                        const uint64_t *row = A + (size_t)k * W;
                        cost += getbit(row, n) ^ getbit(row, T[a]) ^ getbit(row, T[b]);
                    }
                    if (cost < best_cost) { best_cost = cost; best_a = a; best_b = b; }
                }
        }
        /* e' = (e_S, t), mapped back through pi */
        for (int k = 0; k < rank; ++k) {
            const uint64_t *row = A + (size_t)k * W;
            int x = getbit(row, n);
            if (best_a >= 0) x ^= getbit(row, T[best_a]);
            if (best_b >= 0) x ^= getbit(row, T[best_b]);
            eperm[pivcol[k]] = (uint8_t)x;
        }
        if (best_a >= 0) eperm[T[best_a]] = 1;
        if (best_b >= 0) eperm[T[best_b]] = 1;
        for (int j = 0; j < n; ++j) ehat[pi[j]] = eperm[j];
    }
done:
    free(kc); free(pos); free(pi); free(A); free(tmp); free(pivcol); free(isbasis); free(T); free(eperm);
    return ret;
}

/* ------------------------------------------------------------ entry points */

static int build_code(int m, int n, const int32_t *rp, const int32_t *ci, ocode *C) {
    if (m < 0 || n < 0 || rp[0] != 0) return -1;
    for (int c = 0; c < m; ++c) {
        if (rp[c + 1] <= rp[c]) return -1; /* empty or malformed row */
        for (int e = rp[c]; e < rp[c + 1]; ++e) {
            if (ci[e] < 0 || ci[e] >= n) return -1;
            if (e > rp[c] && ci[e] <= ci[e - 1]) return -1;
        }
    }
    C->m = m; C->n = n; C->nnz = rp[m]; C->rp = rp; C->ci = ci;
    C->cp = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    C->cr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(C->nnz > 0 ? C->nnz : 1));
    C->ce = (int32_t *)malloc(sizeof(int32_t) * (size_t)(C->nnz > 0 ? C->nnz : 1));
    for (int e = 0; e < C->nnz; ++e) C->cp[ci[e] + 1]++;
    for (int v = 0; v < n; ++v) C->cp[v + 1] += C->cp[v];
    int *fill = (int *)calloc((size_t)n + 1, sizeof(int));
    for (int c = 0; c < m; ++c) /* rows visited in ascending order => entries ascending by row */
        for (int e = rp[c]; e < rp[c + 1]; ++e) {
            int v = ci[e], t = C->cp[v] + fill[v]++;
            C->cr[t] = c;
            C->ce[t] = e;
        }
    free(fill);
    return 0;
}

static void free_code(ocode *C) { free(C->cp); free(C->cr); free(C->ce); }

typedef struct {
    const ocode *C;
    const orc_params *P;
    const double *prior;
    int64_t lo, hi;
    uint64_t first_shot_id;
    const uint32_t *synd;
    uint32_t *corr;
    uint8_t *flags;
    int32_t *iters;
    double *llr_out;
} job;

static void *run_job(void *arg) {
    job *J = (job *)arg;
    const ocode *C = J->C;
    const int m = C->m, n = C->n, mw = (m + 31) / 32, nw = (n + 31) / 32;
    work W;
    size_t ne = (size_t)(C->nnz > 0 ? C->nnz : 1);
    W.mu = malloc(sizeof(double) * (size_t)(n + 1)); W.lam = malloc(sizeof(double) * (size_t)(n + 1));
    W.alpha = malloc(sizeof(double) * ne); W.beta = malloc(sizeof(double) * ne);
    W.imu = malloc(sizeof(long) * (size_t)(n + 1)); W.ilam = malloc(sizeof(long) * (size_t)(n + 1));
    W.ialpha = malloc(sizeof(long) * ne); W.ibeta = malloc(sizeof(long) * ne);
    W.shat = calloc((size_t)m + 1, 1); W.sprev = calloc((size_t)m + 1, 1);
    W.ulist = malloc(sizeof(int) * (size_t)(m + 1));
    uint8_t *s = malloc((size_t)m + 1), *ehat = malloc((size_t)n + 1), *eosd = malloc((size_t)n + 1);
    double *lam = malloc(sizeof(double) * (size_t)(n + 1));
    for (int64_t k = J->lo; k < J->hi; ++k) {
        const uint32_t *sw = J->synd + k * mw;
        for (int c = 0; c < m; ++c) s[c] = (uint8_t)((sw[c >> 5] >> (c & 31)) & 1u);
        int it = 0, conv = 0;
        uint64_t shot_id = J->first_shot_id + (uint64_t)k;
        memset(W.sprev, 0, (size_t)m);
        if (J->P->msg == ORC_INT8) bp_int8(C, J->P, J->prior, shot_id, s, ehat, &it, &conv, lam, &W);
        else bp_float(C, J->P, J->prior, shot_id, s, ehat, &it, &conv, lam, &W);
        uint8_t fl = conv ? ORC_FLAG_CONVERGED : 0;
        if (!conv && J->P->osd != ORC_OSD_NONE) {
            fl |= ORC_FLAG_OSD;
            if (osd_shot(C, J->P->osd, J->P->osd_order, lam, s, eosd) == 0) memcpy(ehat, eosd, (size_t)n);
            else fl |= ORC_FLAG_OSD_INCONSISTENT;
        }
        uint32_t *cw = J->corr + k * nw;
        memset(cw, 0, sizeof(uint32_t) * (size_t)nw);
        for (int v = 0; v < n; ++v)
            if (ehat[v]) cw[v >> 5] |= 1u << (v & 31);
        if (J->flags) J->flags[k] = fl;
        if (J->iters) J->iters[k] = it;
        if (J->llr_out) memcpy(J->llr_out + k * n, lam, sizeof(double) * (size_t)n);
    }
    free(W.mu); free(W.lam); free(W.alpha); free(W.beta); free(W.imu); free(W.ilam); free(W.ialpha);
    free(W.ibeta); free(W.shat); free(W.sprev); free(W.ulist); free(s); free(ehat); free(eosd); free(lam);
    return NULL;
}

/* Decode n_shots syndromes (packed LSB-first, ceil(m/32) words per shot).
 * Outputs: corrections (ceil(n/32) words per shot), flags, iterations and the
 * lambda of the last BP iteration ([n_shots][n], may be NULL).
 * Returns 0, or -1 for invalid input. */
int orc_decode(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *prior,
               const orc_params *P, int64_t n_shots, uint64_t first_shot_id, const uint32_t *synd,
               uint32_t *corr, uint8_t *flags, int32_t *iters, double *llr_out, int32_t n_threads) {
    ocode C;
    if (P->max_iter < 1 || P->msg < 0 || P->msg > 3) return -1;
    for (int v = 0; v < n; ++v)
        if (!(prior[v] > 0.0 && prior[v] < 1.0)) return -1;
    if (P->msg == ORC_INT8 && (P->fx_int | P->fx_frac) &&
        (P->fx_int < 0 || P->fx_frac < 0 || P->fx_int + P->fx_frac < 1 || P->fx_int + P->fx_frac > 7))
        return -1;
    if (P->msg == ORC_INT8 && P->scale_mode == 1) {
        double k = P->scale * 8.0;
        if (fabs(k - nearbyint(k)) > 1e-12 || k < 1 || k > 8) return -1;
    }
    if (build_code(m, n, row_ptr, col_idx, &C) != 0) return -1;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    if ((int64_t)n_threads > n_shots) n_threads = (int32_t)(n_shots > 0 ? n_shots : 1);
    job jobs[256];
    pthread_t th[256];
    for (int t = 0; t < n_threads; ++t) {
        jobs[t] = (job){&C, P, prior, n_shots * t / n_threads, n_shots * (t + 1) / n_threads, first_shot_id,
                        synd, corr, flags, iters, llr_out};
        if (n_threads == 1) run_job(&jobs[t]);
        else pthread_create(&th[t], NULL, run_job, &jobs[t]);
    }
    if (n_threads > 1)
        for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    free_code(&C);
    return 0;
}

/* The lottery selection (Algorithm 3) on its own, for hand-traced tests:
 * s, sprev: m bytes; lam: n values (Int3.4 when is_int8).  Returns v* or -1. */
int orc_lottery_pick(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, uint64_t seed,
                     uint64_t shot_id, int32_t i, const uint8_t *s, const uint8_t *sprev, const double *lam,
                     int32_t is_int8, int32_t policy, const uint8_t *ehat) {
    ocode C;
    if (build_code(m, n, row_ptr, col_idx, &C) != 0) return -2;
    orc_params P;
    memset(&P, 0, sizeof P);
    P.seed = seed;
    P.policy = policy;
    int *ulist = malloc(sizeof(int) * (size_t)(m + 1));
    long *li = malloc(sizeof(long) * (size_t)(n + 1));
    for (int v = 0; v < n; ++v) li[v] = (long)lam[v];
    int r = lottery_pick(&C, &P, shot_id, i, s, sprev, ulist, is_int8 ? NULL : lam, is_int8 ? li : NULL, ehat);
    free(ulist); free(li);
    free_code(&C);
    return r;
}

/* OSD of one shot given lambda (e.g. the GPU's own lambda).  mode 1 = OSD-0,
 * 2 = OSD-CS(order).  Writes ceil(n/32) correction words and the flag byte
 * (ORC_FLAG_OSD, plus ORC_FLAG_OSD_INCONSISTENT when s is not in the column
 * space; the correction words are then left untouched). */
int orc_osd(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t mode, int32_t order,
            const double *lam, const uint32_t *synd, uint32_t *corr, uint8_t *flag) {
    ocode C;
    if (build_code(m, n, row_ptr, col_idx, &C) != 0) return -1;
    uint8_t *s = malloc((size_t)m + 1), *e = calloc((size_t)n + 1, 1);
    for (int c = 0; c < m; ++c) s[c] = (uint8_t)((synd[c >> 5] >> (c & 31)) & 1u);
    int r = osd_shot(&C, mode, order, lam, s, e);
    *flag = ORC_FLAG_OSD | (r ? ORC_FLAG_OSD_INCONSISTENT : 0);
    if (!r) {
        int nw = (n + 31) / 32;
        memset(corr, 0, sizeof(uint32_t) * (size_t)nw);
        for (int v = 0; v < n; ++v)
            if (e[v]) corr[v >> 5] |= 1u << (v & 31);
    }
    free(s); free(e);
    free_code(&C);
    return 0;
}
