/*
 * psl_oracle.c -- CPU oracle for the two-phase PSL search.
 *
 * TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the bench's
 * CPU-baseline leg are the only code that may load this library. The product
 * library (libpsl) never links, loads or calls it, and the two share no code,
 * header, table or helper.
 *
 * What it follows (Bosković & Brest, "Two-phase optimization of binary
 * sequences with low peak sidelobe level value", arXiv 2107.09801):
 *   Eq. (1)  a sequence of L elements, each +1 or -1;
 *   Eq. (2)  aperiodic autocorrelation C_k = sum_{i=1}^{L-k} s_i s_{i+k};
 *   Eq. (3)  PSL = max |C_k| over the sidelobes;
 *   Eq. (5)  fitness F = sum_{k=1}^{L-1} |C_k|^alpha;
 *   Algorithm 1 (Search) with the Section 3 text: a limited neighbourhood of
 *   N_lmt consecutive single-element flips after a random start, move to the
 *   best neighbour even if worse, keep the best-PSL neighbour, count
 *   unimproved steps and switch phase (exponent) with FLIP_lmt random flips
 *   of the phase's local best.
 *
 * Everything is plain loops in the order the paper states them, with FP64
 * for the fitness. Readings taken where the paper is silent or ambiguous:
 *   R1  indices are 0-based: s[i] is the paper's s_{i+1}; C[k] for k in [0,L).
 *   R2  PSL runs over 1 <= k <= L-1 (Eq. (3) is printed with a strict lower
 *       bound, which would drop k = 1 and make L = 2 degenerate; the fitness
 *       sum of Eq. (5) starts at k = 1).
 *   R3  alpha is an integer in [1,16]; the per-|c| power table is the
 *       left-to-right FP64 product c*c*...*c (alpha factors, each rounded to
 *       nearest even), T[0] = 0.
 *   R4  F is summed in k order with Neumaier's compensated summation.
 *   R5  best-neighbour choice: with F_min the minimum over the scanned
 *       neighbours, the move is the first neighbour in scan order whose
 *       F <= F_min*(1+tau), tau = 1e-12. With only exact ties in the band this
 *       is the strict-less-than scan of Algorithm 1.
 *   R6  improvement test: improved iff v_step < v_local*(1-tau); worse iff
 *       v_step > v_local*(1+tau); otherwise equal (no bookkeeping change).
 *   R7  psl_best starts at the initial pivot's PSL with solution_best = the
 *       initial pivot; local_best starts at the initial pivot and is not
 *       reassigned at a switch.
 *   R8  Rand_flip flips FLIP_lmt distinct positions: positions are drawn as
 *       r mod L, and a repeat is skipped.
 *   R9  random numbers: counter-based SplitMix64 (Steele, Lea & Flood, 2014).
 *       draw(seed, ctr) is output number ctr+1 of the SplitMix64 stream whose
 *       state starts at seed: mix(seed + (ctr+1) * 0x9E3779B97F4A7C15).
 *       Counter tags in bits 63..60: 0 = initial pivot word w (ctr = w);
 *       1 = start of step t (ctr = 1<<60 | t); 2 = switch q, attempt r
 *       (ctr = 2<<60 | q<<24 | r). The initial pivot takes bit (i mod 64) of
 *       word floor(i/64) as element i, bit 1 meaning -1. start = draw mod L.
 *   R10 switch trigger: switch_period == 0 is the paper's rule (unimproved
 *       exceeds LS_lmt); switch_period P > 0 switches after the bookkeeping of
 *       step t whenever (t+1) mod P == 0, with the same switch body.
 *   R11 F of the initial pivot uses alpha_1; after a switch the pivot's F in
 *       the new exponent becomes v_local.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OC_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------ RNG (R9) */

OC_API uint64_t oc_draw(uint64_t seed, uint64_t ctr)
{
    uint64_t z = seed + (ctr + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Rand(L, SEED) of Algorithm 1: the random initial pivot (R9). */
OC_API void oc_rand_pivot(uint64_t seed, int L, int8_t *s)
{
    for (int i = 0; i < L; ++i) {
        uint64_t word = oc_draw(seed, (uint64_t)(i / 64));
        int bit = (int)((word >> (i % 64)) & 1u);
        s[i] = bit ? -1 : +1;
    }
}

/* Conversions between the +-1 form and the packed form used at the library
 * boundary (64-bit words, element i in bit i%64 of word i/64, 1 = -1). */
OC_API void oc_bits_to_seq(const uint64_t *bits, int L, int8_t *s)
{
    for (int i = 0; i < L; ++i)
        s[i] = ((bits[i / 64] >> (i % 64)) & 1u) ? -1 : +1;
}

OC_API void oc_seq_to_bits(const int8_t *s, int L, uint64_t *bits)
{
    int nw = (L + 63) / 64;
    for (int w = 0; w < nw; ++w) bits[w] = 0;
    for (int i = 0; i < L; ++i)
        if (s[i] < 0) bits[i / 64] |= (uint64_t)1 << (i % 64);
}

/* ------------------------------------------------------- Eq. (2), Eq. (3) */

/* Aperiodic autocorrelation by its definition, O(L^2). Long sequences spread
 * the shifts k over threads; each C_k is an integer sum, so its value does
 * not depend on how the shifts are divided. */
OC_API void oc_corr(const int8_t *s, int L, int32_t *C)
{
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 256) if (L >= 8192)
#endif
    for (int k = 0; k < L; ++k) {
        int32_t acc = 0;
        for (int i = 0; i + k < L; ++i)
            acc += (int32_t)s[i] * (int32_t)s[i + k];
        C[k] = acc;
    }
}

/* Peak sidelobe level, k = 1..L-1 (R2). */
OC_API int32_t oc_psl(const int32_t *C, int L)
{
    int32_t m = 0;
    for (int k = 1; k < L; ++k) {
        int32_t a = C[k] < 0 ? -C[k] : C[k];
        if (a > m) m = a;
    }
    return m;
}

/* ------------------------------------------------------------- Eq. (5) */

/* Per-|c| power table (R3): T[c] = c^alpha as a left-to-right FP64 product. */
OC_API void oc_power_table(int alpha, int n, double *T)
{
    for (int c = 0; c < n; ++c) {
        double p = (double)c;
        for (int a = 1; a < alpha; ++a) p = p * (double)c;
        T[c] = p;
    }
}

/* Neumaier's compensated summation, one term at a time (R4). */
typedef struct { double sum, comp; } oc_nsum;

static void nsum_add(oc_nsum *a, double x)
{
    double t = a->sum + x;
    double as = a->sum < 0 ? -a->sum : a->sum;
    double ax = x < 0 ? -x : x;
    if (as >= ax) a->comp += (a->sum - t) + x;
    else          a->comp += (x - t) + a->sum;
    a->sum = t;
}

static double nsum_get(const oc_nsum *a) { return a->sum + a->comp; }

/* Fitness of Eq. (5) from C and the power table. */
OC_API double oc_fitness(const int32_t *C, int L, const double *T)
{
    oc_nsum acc = {0.0, 0.0};
    for (int k = 1; k < L; ++k) {
        int32_t a = C[k] < 0 ? -C[k] : C[k];
        nsum_add(&acc, T[a]);
    }
    return nsum_get(&acc);
}

/* ------------------------------------------- one-element flip (Section 3) */

/* Neighbour correlations, definition tier: flip element j, recompute Eq. (2). */
OC_API void oc_flip_corr_definition(const int8_t *s, int L, int j, int32_t *Cn)
{
    int8_t *t = (int8_t *)malloc((size_t)L);
    memcpy(t, s, (size_t)L);
    t[j] = (int8_t)-t[j];
    oc_corr(t, L, Cn);
    free(t);
}

/* Neighbour correlations, formula tier. Flipping s_j changes exactly the two
 * products of Eq. (2) that contain s_j at shift k, s_j*s_{j+k} and
 * s_{j-k}*s_j, when those indices exist; each changes sign, so
 * C'_k = C_k - 2 s_j (s_{j+k}[j+k<L] + s_{j-k}[j-k>=0]). */
OC_API void oc_flip_corr_formula(const int8_t *s, const int32_t *C, int L, int j,
                                 int32_t *Cn)
{
    Cn[0] = C[0];
    for (int k = 1; k < L; ++k) {
        int32_t d = 0;
        if (j + k < L) d += s[j + k];
        if (j - k >= 0) d += s[j - k];
        Cn[k] = C[k] - 2 * (int32_t)s[j] * d;
    }
}

/* Neighborhood(pivot, f, alpha, N_lmt, start) of Algorithm 1: F and PSL of
 * the neighbours j = (start + i) mod L, i = 1..n_lmt; entry i-1 is neighbour
 * i. Each neighbour is the formula tier written out one shift at a time.
 * The loop over neighbours may run on several threads; each neighbour's
 * arithmetic is the same on any thread count. */
OC_API void oc_eval_neighbourhood(const int8_t *s, const int32_t *C, int L,
                                  const double *T, uint32_t start, uint32_t n_lmt,
                                  double *F, int32_t *P, int nthreads)
{
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (int64_t i = 1; i <= (int64_t)n_lmt; ++i) {
        int j = (int)(((uint64_t)start + (uint64_t)i) % (uint64_t)L);
        oc_nsum acc = {0.0, 0.0};
        int32_t peak = 0;
        for (int k = 1; k < L; ++k) {
            int32_t d = 0;
            if (j + k < L) d += s[j + k];
            if (j - k >= 0) d += s[j - k];
            int32_t c = C[k] - 2 * (int32_t)s[j] * d;
            int32_t a = c < 0 ? -c : c;
            nsum_add(&acc, T[a]);
            if (a > peak) peak = a;
        }
        F[i - 1] = nsum_get(&acc);
        P[i - 1] = peak;
    }
}

/* ------------------------------------------------ selection (R5, Alg. 1) */

enum {
    OC_AMBIG_ARGMIN = 1,   /* some F lies within margin*F_min of the band edge */
    OC_AMBIG_COMPARE = 2,  /* v_step/v_local lies within margin of 1 -+ tau   */
    OC_IMPROVED = 4,
    OC_WORSE = 8,
    OC_SWITCHED = 16,
    OC_PSL_IMPROVED = 32,
    OC_SELFCHECK_FAILED = 64,  /* C broke an identity of Eq. (2), or differs
                                  from a from-scratch recomputation */
};

typedef struct {
    uint32_t i_best;   /* scan index (0-based) of the chosen move */
    double   F_best;   /* its F                                     */
    double   F_min;    /* minimum F over the scan                   */
    uint32_t i_psl;    /* first scan index with the minimum PSL     */
    int32_t  psl_min;  /* that PSL                                  */
    uint32_t flags;    /* OC_AMBIG_ARGMIN                           */
} oc_choice;

OC_API void oc_select(const double *F, const int32_t *P, uint32_t n, double tau,
                      double margin, oc_choice *out)
{
    double fmin = F[0];
    for (uint32_t i = 1; i < n; ++i)
        if (F[i] < fmin) fmin = F[i];
    double thr = fmin * (1.0 + tau);
    uint32_t ib = 0;
    int found = 0;
    uint32_t flags = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (!found && F[i] <= thr) { ib = i; found = 1; }
        double gap = F[i] - thr;
        if (gap < 0) gap = -gap;
        if (gap <= margin * fmin) flags |= OC_AMBIG_ARGMIN;
    }
    int32_t pmin = P[0];
    uint32_t ip = 0;
    for (uint32_t i = 1; i < n; ++i)
        if (P[i] < pmin) { pmin = P[i]; ip = i; }
    out->i_best = ib;
    out->F_best = F[ib];
    out->F_min = fmin;
    out->i_psl = ip;
    out->psl_min = pmin;
    out->flags = flags;
}

/* ------------------------------------------------------ Algorithm 1 walk */

typedef struct {
    /* control parameters (Section 4.1) */
    int L;
    uint64_t seed;
    int alpha1, alpha2;
    uint32_t n_lmt, ls_lmt, flip_lmt, switch_period;
    /* state */
    int8_t *pivot, *local_best, *solution_best;
    int32_t *C;
    int alpha;            /* current exponent */
    double value_local;
    int32_t psl_best;
    uint32_t unimproved;
    uint64_t t;           /* steps done */
    uint64_t q;           /* switches done */
    double F_pivot;       /* F of the pivot in the current exponent */
    int32_t psl_pivot;
    double *T1, *T2;      /* power tables for alpha1 and alpha2, |c| <= L */
    double *F;
    int32_t *P;
} oc_walk;

typedef struct {
    uint32_t start;
    uint32_t k;           /* the move (element index) */
    double   value_step;  /* F of the move */
    double   F_min;
    int32_t  psl_k;       /* PSL of the move */
    uint32_t j_psl;       /* element index of the best-PSL neighbour */
    int32_t  psl_min;
    int32_t  psl_best;    /* after the step */
    int32_t  alpha;       /* after the step */
    uint32_t unimproved;  /* after the step */
    double   value_local; /* after the step */
    uint32_t flags;
} oc_trace;

static const double *walk_table(const oc_walk *w)
{
    return w->alpha == w->alpha1 ? w->T1 : w->T2;
}

OC_API void oc_walk_destroy(oc_walk *w)
{
    if (!w) return;
    free(w->pivot); free(w->local_best); free(w->solution_best);
    free(w->C); free(w->T1); free(w->T2); free(w->F); free(w->P);
    free(w);
}

/* Lines before the while loop of Algorithm 1: the pivot (random, or given),
 * its correlations and F in alpha_1, and the initial bests (R7, R11). */
OC_API oc_walk *oc_walk_create(int L, uint64_t seed, int alpha1, int alpha2,
                               uint32_t n_lmt, uint32_t ls_lmt, uint32_t flip_lmt,
                               uint32_t switch_period, const uint64_t *init_bits)
{
    if (L < 2 || alpha1 < 1 || alpha2 < 1 || alpha1 > 16 || alpha2 > 16) return NULL;
    if (n_lmt < 1 || n_lmt > (uint32_t)L || flip_lmt > (uint32_t)L) return NULL;
    oc_walk *w = (oc_walk *)calloc(1, sizeof(oc_walk));
    w->L = L; w->seed = seed; w->alpha1 = alpha1; w->alpha2 = alpha2;
    w->n_lmt = n_lmt; w->ls_lmt = ls_lmt; w->flip_lmt = flip_lmt;
    w->switch_period = switch_period;
    w->pivot = (int8_t *)malloc((size_t)L);
    w->local_best = (int8_t *)malloc((size_t)L);
    w->solution_best = (int8_t *)malloc((size_t)L);
    w->C = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
    w->T1 = (double *)malloc(sizeof(double) * (size_t)(L + 1));
    w->T2 = (double *)malloc(sizeof(double) * (size_t)(L + 1));
    w->F = (double *)malloc(sizeof(double) * (size_t)L);
    w->P = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
    oc_power_table(alpha1, L + 1, w->T1);
    oc_power_table(alpha2, L + 1, w->T2);
    if (init_bits) oc_bits_to_seq(init_bits, L, w->pivot);
    else           oc_rand_pivot(seed, L, w->pivot);
    oc_corr(w->pivot, L, w->C);
    w->alpha = alpha1;
    w->value_local = oc_fitness(w->C, L, walk_table(w));
    w->F_pivot = w->value_local;
    w->psl_pivot = oc_psl(w->C, L);
    w->psl_best = w->psl_pivot;
    memcpy(w->local_best, w->pivot, (size_t)L);
    memcpy(w->solution_best, w->pivot, (size_t)L);
    return w;
}

/* Phase switch: Rand_flip of the local best (R8), exponent swap, Fitness. */
static void walk_switch(oc_walk *w)
{
    int L = w->L;
    memcpy(w->pivot, w->local_best, (size_t)L);
    uint8_t *chosen = (uint8_t *)calloc((size_t)L, 1);
    uint32_t done = 0;
    for (uint64_t r = 0; done < w->flip_lmt; ++r) {
        uint64_t ctr = (2ull << 60) | (w->q << 24) | r;
        uint32_t pos = (uint32_t)(oc_draw(w->seed, ctr) % (uint64_t)L);
        if (chosen[pos]) continue;
        chosen[pos] = 1;
        w->pivot[pos] = (int8_t)-w->pivot[pos];
        ++done;
    }
    free(chosen);
    w->alpha = (w->alpha == w->alpha1) ? w->alpha2 : w->alpha1;
    oc_corr(w->pivot, L, w->C);
    w->value_local = oc_fitness(w->C, L, walk_table(w));
    w->F_pivot = w->value_local;
    w->psl_pivot = oc_psl(w->C, L);
    w->unimproved = 0;
    w->q += 1;
}

/* Identities every C of Eq. (2) satisfies: C_0 = L; C_{L-1} = s_0 s_{L-1};
 * C_k has the parity of L-k and |C_k| <= L-k; (sum s)^2 = L + 2 sum_{k>=1} C_k
 * (square the sum and group the products by their distance). With `full`,
 * C is also compared with Eq. (2) recomputed from the sequence. Returns 1 if
 * all hold. */
OC_API int oc_check_corr(const int8_t *s, const int32_t *C, int L, int full)
{
    if (C[0] != L || C[L - 1] != (int32_t)s[0] * (int32_t)s[L - 1]) return 0;
    int64_t sum_s = 0, sum_c = 0;
    for (int i = 0; i < L; ++i) sum_s += s[i];
    for (int k = 1; k < L; ++k) {
        int64_t c = C[k], room = L - k;
        if (c > room || c < -room || ((c - room) % 2) != 0) return 0;
        sum_c += c;
    }
    if (sum_s * sum_s != (int64_t)L + 2 * sum_c) return 0;
    if (full) {
        int32_t *R = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
        oc_corr(s, L, R);
        int same = memcmp(R, C, sizeof(int32_t) * (size_t)L) == 0;
        free(R);
        if (!same) return 0;
    }
    return 1;
}

static int walk_check_corr(const oc_walk *w, int full)
{
    return oc_check_corr(w->pivot, w->C, w->L, full);
}

/* One iteration of the while loop of Algorithm 1. `force_k` >= 0 replaces
 * the chosen move (used only to follow a decision taken elsewhere). After the
 * step the walk checks its C against the identities of Eq. (2), and every
 * 64 steps against a from-scratch recomputation; a failure sets
 * OC_SELFCHECK_FAILED. */
OC_API void oc_walk_step(oc_walk *w, double tau, double margin, int nthreads,
                         int32_t force_k, oc_trace *tr)
{
    int L = w->L;
    uint32_t start = (uint32_t)(oc_draw(w->seed, (1ull << 60) | w->t) % (uint64_t)L);
    oc_eval_neighbourhood(w->pivot, w->C, L, walk_table(w), start, w->n_lmt,
                          w->F, w->P, nthreads);
    oc_choice ch;
    oc_select(w->F, w->P, w->n_lmt, tau, margin, &ch);
    uint32_t flags = ch.flags;
    uint32_t ib = ch.i_best;
    uint32_t k = (uint32_t)((start + ib + 1u) % (uint32_t)L);
    if (force_k >= 0) {
        /* scan index of the forced element */
        k = (uint32_t)force_k;
        ib = (uint32_t)(((uint64_t)k + 2u * (uint64_t)L - start - 1u) % (uint64_t)L);
    }
    double value_step = w->F[ib];
    int32_t psl_k = w->P[ib];
    uint32_t j_psl = (uint32_t)((start + ch.i_psl + 1u) % (uint32_t)L);

    /* best-PSL neighbour, strict improvement only */
    if (ch.psl_min < w->psl_best) {
        w->psl_best = ch.psl_min;
        memcpy(w->solution_best, w->pivot, (size_t)L);
        w->solution_best[j_psl] = (int8_t)-w->solution_best[j_psl];
        flags |= OC_PSL_IMPROVED;
    }

    /* Flip(pivot, k): the move, with C updated by the one-element formula */
    {
        int32_t *Cn = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
        oc_flip_corr_formula(w->pivot, w->C, L, (int)k, Cn);
        memcpy(w->C, Cn, sizeof(int32_t) * (size_t)L);
        free(Cn);
        w->pivot[k] = (int8_t)-w->pivot[k];
        w->F_pivot = value_step;
        w->psl_pivot = psl_k;
    }

    /* three-way comparison with the local best (R6) */
    double lo = w->value_local * (1.0 - tau), hi = w->value_local * (1.0 + tau);
    double band = margin * w->value_local;
    if ((value_step - lo < band && lo - value_step < band) ||
        (value_step - hi < band && hi - value_step < band))
        flags |= OC_AMBIG_COMPARE;
    if (value_step < lo) {
        w->unimproved = 0;
        memcpy(w->local_best, w->pivot, (size_t)L);
        w->value_local = value_step;
        flags |= OC_IMPROVED;
    } else if (value_step > hi) {
        w->unimproved += 1;
        flags |= OC_WORSE;
        if (w->switch_period == 0 && w->unimproved > w->ls_lmt) {
            walk_switch(w);
            flags |= OC_SWITCHED;
        }
    }
    if (w->switch_period > 0 && ((w->t + 1) % w->switch_period) == 0) {
        walk_switch(w);
        flags |= OC_SWITCHED;
    }
    w->t += 1;
    if (!walk_check_corr(w, (w->t % 64) == 0)) flags |= OC_SELFCHECK_FAILED;

    if (tr) {
        tr->start = start;
        tr->k = k;
        tr->value_step = value_step;
        tr->F_min = ch.F_min;
        tr->psl_k = psl_k;
        tr->j_psl = j_psl;
        tr->psl_min = ch.psl_min;
        tr->psl_best = w->psl_best;
        tr->alpha = w->alpha;
        tr->unimproved = w->unimproved;
        tr->value_local = w->value_local;
        tr->flags = flags;
    }
}

/* Read back the walk: packed pivot, local best and best-PSL sequences, C and
 * the scalars. Any pointer may be NULL. */
OC_API void oc_walk_read(const oc_walk *w, uint64_t *pivot_bits, uint64_t *local_best_bits,
                         uint64_t *best_bits, int32_t *C, double *scalars_f,
                         int64_t *scalars_i)
{
    int L = w->L;
    if (pivot_bits) oc_seq_to_bits(w->pivot, L, pivot_bits);
    if (local_best_bits) oc_seq_to_bits(w->local_best, L, local_best_bits);
    if (best_bits) oc_seq_to_bits(w->solution_best, L, best_bits);
    if (C) memcpy(C, w->C, sizeof(int32_t) * (size_t)L);
    if (scalars_f) {
        scalars_f[0] = w->value_local;
        scalars_f[1] = w->F_pivot;
    }
    if (scalars_i) {
        scalars_i[0] = w->alpha;
        scalars_i[1] = w->psl_best;
        scalars_i[2] = w->unimproved;
        scalars_i[3] = (int64_t)w->t;
        scalars_i[4] = (int64_t)w->q;
        scalars_i[5] = w->psl_pivot;
    }
}

/* The last neighbourhood's F and PSL arrays (n_lmt entries, scan order). */
OC_API void oc_walk_last_neighbourhood(const oc_walk *w, double *F, int32_t *P)
{
    if (F) memcpy(F, w->F, sizeof(double) * w->n_lmt);
    if (P) memcpy(P, w->P, sizeof(int32_t) * w->n_lmt);
}

/* -------------------------------------------- Eq. (4) by brute force */

/* Minimum PSL over all 2^(L-1) sequences with s_1 = +1 (a sign change of the
 * whole sequence leaves every C_k unchanged), by the definition of Eq. (2).
 * count_out receives the number of sequences (with s_1 = +1) that reach it. */
OC_API int32_t oc_min_psl_bruteforce(int L, uint64_t *count_out, int nthreads)
{
    if (L < 2 || L > 30) return -1;
    uint64_t n = 1ull << (L - 1);
    int32_t best = L;
    uint64_t count = 0;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
#endif
    {
        int32_t lbest = L;
        uint64_t lcount = 0;
        int8_t s[32];
        int32_t C[32];
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int64_t m = 0; m < (int64_t)n; ++m) {
            s[0] = +1;
            for (int i = 1; i < L; ++i) s[i] = ((m >> (i - 1)) & 1) ? -1 : +1;
            oc_corr(s, L, C);
            int32_t p = oc_psl(C, L);
            if (p < lbest) { lbest = p; lcount = 1; }
            else if (p == lbest) ++lcount;
        }
#ifdef _OPENMP
#pragma omp critical
#endif
        {
            if (lbest < best) { best = lbest; count = lcount; }
            else if (lbest == best) count += lcount;
        }
    }
    if (count_out) *count_out = count;
    return best;
}

OC_API int oc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
