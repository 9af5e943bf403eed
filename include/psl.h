/*
 * psl.h -- libpsl: MI355X (gfx950) engine for the data-parallel hot path of
 * the two-phase stochastic search for +-1 sequences with a low peak sidelobe
 * level (Boskovic & Brest, arXiv 2107.09801).
 *
 * Problem statement followed by every call:
 *   Eq. (1)  a sequence S_L of L elements, each +1 or -1;
 *   Eq. (2)  C_k = sum_{i=1}^{L-k} s_i s_{i+k}, k = 0..L-1;
 *   Eq. (3)  PSL = max |C_k| over the sidelobes k = 1..L-1;
 *   Eq. (5)  F = sum_{k=1}^{L-1} |C_k|^alpha, alpha the current phase's
 *            exponent;
 *   Algorithm 1 (Search) and the Section 3 text: the limited neighbourhood,
 *   the move to the best neighbour, best-PSL tracking, the unimproved
 *   counter and the phase switch (Rand_flip of the local best, exponent swap).
 *
 * Conventions
 *   Indices are 0-based: element i is the paper's s_{i+1}; C[k] for k in
 *   [0, L). Sequences cross the boundary packed: ceil(L/64) 64-bit words,
 *   element i in bit (i % 64) of word i/64, bit 1 meaning -1, bits at and
 *   beyond L zero.
 *   Every call returns a psl_status. Nothing throws or aborts across the
 *   boundary. Errors from asynchronous device work surface at the next call
 *   that synchronises (psl_sync, psl_read_walk, psl_eval_neighbourhood, ...).
 *   A context is used by one host thread at a time, except the psl_serve_*
 *   calls, which are thread-safe.
 *   All device memory a context uses is owned by the context. Pointers
 *   documented as device pointers are caller-owned device memory on the
 *   context's device; host pointers are caller-owned host memory.
 *
 * Readings where the paper is silent or ambiguous (shared with the tests):
 *   - PSL runs over 1 <= k <= L-1.
 *   - alpha is an integer in [1,16]; |c|^alpha comes from a per-|c| FP64
 *     table whose entry is the left-to-right product c*c*...*c.
 *   - Best-neighbour choice: the first neighbour in scan order whose F lies
 *     within F_min*(1+tau) of the minimum, tau = 1e-12 (the strict-less-than
 *     scan of Algorithm 1 when the band holds only exact ties).
 *   - Improvement test: improved iff v_step < v_local*(1-tau), worse iff
 *     v_step > v_local*(1+tau), otherwise no bookkeeping change.
 *   - psl_best starts at the initial pivot's PSL (the best sequence is the
 *     initial pivot); local_best starts at the initial pivot and is not
 *     reassigned at a switch.
 *   - Rand_flip flips FLIP_lmt distinct positions (draw r mod L, skip
 *     repeats, FLIP_lmt <= 1024).
 *   - Random numbers are counter-based SplitMix64 (Steele, Lea & Flood 2014):
 *     draw(seed, ctr) = mix(seed + (ctr+1)*0x9E3779B97F4A7C15). Counters:
 *     initial pivot word w -> w; start of step t -> (1<<60)|t; switch q,
 *     attempt r -> (2<<60)|(q<<24)|r. Element i of a random initial pivot
 *     is bit (i%64) of draw(seed, i/64). start = draw mod L.
 *   - switch_period 0 is the paper's trigger (unimproved > LS_lmt); P > 0
 *     switches after the bookkeeping of step t whenever (t+1) mod P == 0.
 */
#ifndef PSL_H
#define PSL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define PSL_API __attribute__((visibility("default")))
#else
#define PSL_API
#endif

typedef int32_t psl_status;
#define PSL_OK        0
#define PSL_E_INVAL  (-1)   /* an argument is out of range or inconsistent  */
#define PSL_E_NOMEM  (-2)   /* device memory (or the arena) is exhausted     */
#define PSL_E_HIP    (-3)   /* a HIP runtime call or kernel failed           */
#define PSL_E_STATE  (-4)   /* unknown walk or ticket, or wrong call order   */
#define PSL_E_AGAIN  (-5)   /* serving: the job is queued or running         */
#define PSL_E_FULL   (-6)   /* serving: the job can never fit the budget     */

#define PSL_L_MAX        1048575u   /* 2^20 - 1, the paper's largest L        */
#define PSL_ALPHA_MAX    16u
#define PSL_FLIP_LMT_MAX 1024u

typedef struct psl_ctx psl_ctx;

/* Control parameters of Search (Algorithm 1; the list in Section 4.1). */
typedef struct {
    uint32_t L;              /* sequence length, 2 <= L <= PSL_L_MAX          */
    uint32_t alpha1;         /* exponent of the first phase, 1..16            */
    uint32_t alpha2;         /* exponent of the second phase, 1..16           */
    uint32_t n_lmt;          /* N_lmt, 1..L; 0 means L (full neighbourhood)   */
    uint32_t ls_lmt;         /* LS_lmt, used when switch_period == 0          */
    uint32_t flip_lmt;       /* FLIP_lmt, 0..min(L, PSL_FLIP_LMT_MAX)         */
    uint32_t switch_period;  /* 0: paper trigger; P > 0: every P steps        */
    uint32_t reserved;       /* must be 0                                     */
    uint64_t seed;           /* SEED of Rand                                  */
} psl_walk_cfg;

/* Result of one limited-neighbourhood evaluation (the scan of Algorithm 1). */
typedef struct {
    uint32_t j_best;    /* element index of the move (best neighbour)         */
    uint32_t i_best;    /* its scan index: j_best = (start + i_best + 1) % L   */
    double   F_best;    /* its F (value_step)                                  */
    double   F_min;     /* the minimum F over the scanned neighbours           */
    uint32_t j_psl;     /* element index of the first neighbour with min PSL  */
    int32_t  psl_min;   /* that PSL                                            */
    int32_t  psl_k;     /* PSL of the move                                     */
    uint32_t flags;     /* PSL_CHOICE_AMBIGUOUS_ARGMIN or 0                    */
} psl_choice;

/* psl_choice.flags: some scanned neighbour's F lies within m*F_min of the
 * band edge F_min*(1+tau) (|F - F_min*(1+tau)| <= m*F_min, m the context's
 * PSL_OPT_AMBIG_MARGIN, 5e-13 by default). Such a move is decided by the
 * rounding of Eq. (5) rather than by the band: an exact summation could put
 * that neighbour on the other side of the edge, so a caller that needs the
 * strict-less-than scan of Algorithm 1 exactly must resolve the step itself
 * (the test suite imposes its CPU oracle's decision). */
#define PSL_CHOICE_AMBIGUOUS_ARGMIN 1u

/* Snapshot of a walk's scalar state. */
typedef struct {
    uint32_t L, alpha1, alpha2, alpha;   /* alpha: the current exponent      */
    uint32_t n_lmt, ls_lmt, flip_lmt, switch_period;
    uint64_t seed;
    uint64_t t;                /* steps done                                  */
    uint64_t q;                /* switches done                               */
    double   value_local;      /* F of the phase's local best                 */
    double   F_pivot;          /* F of the pivot in the current exponent      */
    int32_t  psl_pivot;        /* PSL of the pivot                            */
    int32_t  psl_best;         /* best PSL seen (solution_best's PSL)         */
    uint32_t unimproved;
    uint32_t last_k;           /* element flipped by the last step            */
    double   last_value_step;  /* F of the last move                          */
    uint32_t last_start;       /* start of the last limited neighbourhood     */
    uint32_t last_flags;       /* PSL_STEP_* bits of the last step            */
} psl_walk_state;

#define PSL_STEP_IMPROVED     1u
#define PSL_STEP_WORSE        2u
#define PSL_STEP_SWITCHED     4u
#define PSL_STEP_PSL_IMPROVED 8u
/* The step's best-neighbour choice was ambiguous (as PSL_CHOICE_AMBIGUOUS_ARGMIN). */
#define PSL_STEP_AMBIG_ARGMIN 16u
/* The three-way comparison was ambiguous: the move's F lies strictly within
 * m*v_local of v_local*(1-tau) or of v_local*(1+tau) (m = PSL_OPT_AMBIG_MARGIN). */
#define PSL_STEP_AMBIG_COMPARE 32u

/* ------------------------------------------------------------ context */

/* Create a context on HIP device `device`. `hip_stream` is a hipStream_t to
 * run on (NULL: the context creates its own). If `arena` is non-NULL it is a
 * caller-owned device buffer of `arena_bytes` bytes from which every walk slab
 * is carved (it must outlive the context); otherwise slabs come from hipMalloc.
 * Errors: PSL_E_INVAL (bad device or null out), PSL_E_HIP. */
PSL_API psl_status psl_ctx_create(int device, void *hip_stream, void *arena, size_t arena_bytes,
                          psl_ctx **out);

/* Destroy a context: stops serving, waits for its work, frees its memory. */
PSL_API void psl_ctx_destroy(psl_ctx *ctx);

/* Text of the last error on this context (never NULL; "" if none). */
PSL_API const char *psl_last_error(const psl_ctx *ctx);

/* Wait for all work queued on the context's stream. */
PSL_API psl_status psl_sync(psl_ctx *ctx);

/* ------------------------------------------------------------- walks */

/* Start `n` walks with the same control parameters: the lines of Algorithm 1
 * before its loop. Walk w's pivot is init_bits[w] (host, packed) when
 * init_bits and init_bits[w] are non-NULL, otherwise Rand(L, cfg->seed + w).
 * Computes C (Eq. (2)), F in alpha1 (Eq. (5)) as value_local, the PSL
 * (Eq. (3)) as psl_best; local_best and solution_best start as the pivot.
 * walk_ids_out (host, n entries) receives the walk handles. Blocking.
 * Errors: PSL_E_INVAL (cfg out of range), PSL_E_NOMEM, PSL_E_HIP. */
PSL_API psl_status psl_init_walks(psl_ctx *ctx, const psl_walk_cfg *cfg, uint32_t n,
                          const uint64_t *const *init_bits, uint32_t *walk_ids_out);

/* Release walks (their slabs return to the context). PSL_E_STATE for an
 * unknown handle (the others are still released). */
PSL_API psl_status psl_free_walks(psl_ctx *ctx, const uint32_t *walk_ids, uint32_t n);

/* Neighborhood(pivot, f, alpha, N_lmt, start) of Algorithm 1 for one walk,
 * with the walk's current exponent, followed by the scan that picks the move
 * and the best-PSL neighbour. Pure: the walk is not changed. Entry i-1 of
 * the outputs belongs to element j = (start + i) % L, i = 1..n_lmt
 * (1 <= n_lmt <= L, start < L). F_dev (FP64) and psl_dev (int32) are
 * optional device arrays of n_lmt entries; out (host) receives the choice.
 * Blocking. Errors: PSL_E_INVAL, PSL_E_STATE (unknown walk), PSL_E_HIP. */
PSL_API psl_status psl_eval_neighbourhood(psl_ctx *ctx, uint32_t walk, uint32_t start,
                                  uint32_t n_lmt, double *F_dev, int32_t *psl_dev,
                                  psl_choice *out);

/* psl_eval_neighbourhood for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same evaluation, kernels and results, but every scratch
 * array of the call (work items, k-split partial sums, chunk suffix arrays,
 * near-peak list, combine minima, the choice record) is carved from a fixed
 * 64 MiB device array that each device the library runs on holds until the
 * process ends; the call makes no hipMalloc, hipFree or other device
 * allocation. F_dev and psl_dev are required (caller-owned device memory of
 * n_lmt entries; the kernels write them directly); out is as for
 * psl_eval_neighbourhood. Every call on a device shares that device's array
 * and leaves its contents behind (each call clears what must start at zero
 * with a kernel): calls that overlap on one device, from two contexts or two
 * threads, race. Errors: as psl_eval_neighbourhood; PSL_E_INVAL if F_dev or
 * psl_dev is NULL; PSL_E_NOMEM if the evaluation's scratch would exceed the
 * 64 MiB (the message gives the limit), with nothing launched. */
PSL_API psl_status psl_eval_neighbourhood_noalloc(psl_ctx *ctx, uint32_t walk, uint32_t start,
                                                  uint32_t n_lmt, double *F_dev, int32_t *psl_dev,
                                                  psl_choice *out);

/* Flip(pivot, j) of Algorithm 1: element j changes sign and C is updated in
 * O(L) by the one-element flip C'_k = C_k - 2 s_j (s_{j+k} + s_{j-k}) (terms
 * that stay in bounds only); the pivot's F and PSL are recomputed. No
 * bookkeeping, best tracking or phase logic runs. Blocking.
 * Errors: PSL_E_INVAL (j >= L), PSL_E_STATE, PSL_E_HIP. */
PSL_API psl_status psl_apply_flip(psl_ctx *ctx, uint32_t walk, uint32_t j);

/* Run `steps` iterations of the loop of Algorithm 1 on each of the `n`
 * walks (host array of handles, no repeats): random start, limited
 * neighbourhood, best-neighbour and best-PSL scan, Flip, the three-way
 * comparison and the phase switch. Work is queued on the context's stream;
 * with PSL_STEP_BLOCKING the call waits for it. Walks of different L may be
 * mixed. Errors: PSL_E_INVAL, PSL_E_STATE, PSL_E_NOMEM, PSL_E_HIP. */
#define PSL_STEP_BLOCKING 1u
#define PSL_STEP_GRAPH    2u   /* replay one captured hipGraph per step (the
                                  capture is cached with the batch; ignored
                                  while timing is enabled) */
PSL_API psl_status psl_step_batch(psl_ctx *ctx, const uint32_t *walk_ids, uint32_t n,
                          uint32_t steps, uint32_t flags);

/* Copy a walk to host memory. `out` receives the scalars; pivot_bits,
 * local_best_bits and best_bits (ceil(L/64) words each) and C (L int32) are
 * optional host buffers. Waits for queued work first.
 * Errors: PSL_E_STATE, PSL_E_HIP. */
PSL_API psl_status psl_read_walk(psl_ctx *ctx, uint32_t walk, psl_walk_state *out,
                         uint64_t *pivot_bits, uint64_t *local_best_bits,
                         uint64_t *best_bits, int32_t *C);

/* ----------------------------------------------------------- serving */

/* A request loop on its own host thread: jobs (one walk each, any L, their
 * own step budget) are admitted in arrival order as device memory and slots
 * allow, their walks stay resident in HBM, and every iteration advances every
 * admitted walk by one step of Algorithm 1 in one batched launch sequence
 * (continuous batching: jobs that arrive while others run join the next
 * iteration). While serving, the context's other calls return PSL_E_STATE. */
/* Device memory: the loop's allocations (walk slabs, slabs of finished jobs
 * kept for reuse, scratch buffers) stay within hbm_budget + 1 MiB; a job is
 * admitted while the footprints of the admitted jobs plus the kept slabs fit
 * in hbm_budget. Nothing is allocated before jobs arrive, and a stopped loop
 * holds no device memory (the context's power tables, built by the first
 * start, are the context's). */
typedef struct {
    uint64_t hbm_budget;     /* bytes jobs may occupy: walk slabs and their scratch */
    uint32_t max_slots;      /* most jobs admitted at once (>= 1)                  */
    uint32_t flags;          /* reserved, 0                                         */
} psl_serve_cfg;

typedef struct {
    psl_walk_cfg cfg;        /* the job's walk (cfg.seed is its SEED)              */
    uint64_t step_budget;    /* iterations of Algorithm 1 to run, >= 1              */
    uint64_t *best_bits_out; /* host, ceil(L/64) words, or NULL: receives the best-
                                PSL sequence; must stay valid until the job is
                                polled done                                        */
} psl_job;

typedef struct {
    int32_t  status;         /* PSL_OK; PSL_E_HIP if a device error ended it;
                                PSL_E_STATE if it was cancelled by psl_serve_stop;
                                PSL_E_NOMEM if its slab could not be allocated
                                with no other job admitted                         */
    int32_t  psl_best;       /* best PSL seen                                       */
    int32_t  psl_final;      /* PSL of the final pivot                              */
    uint32_t alpha_final;    /* exponent at the end                                 */
    double   F_final;        /* F of the final pivot in that exponent               */
    uint64_t steps;          /* steps run                                           */
    uint64_t t_arrive_ns;    /* steady-clock times: submit, admit, done             */
    uint64_t t_admit_ns;
    uint64_t t_done_ns;
} psl_job_result;

typedef struct {
    uint64_t submitted, completed, failed, active, queued;
    uint64_t iterations;     /* batched steps launched                              */
    uint64_t flip_evals;     /* neighbour evaluations done                          */
    uint64_t ck_updates;     /* flip_evals x (L-1), nominal                         */
    double   busy_s;         /* wall time with at least one job admitted            */
    uint64_t peak_active;    /* most jobs admitted at once                          */
    uint64_t peak_used;      /* most budget bytes held at once                      */
} psl_serve_stats;

/* Start the loop on this context. Errors: PSL_E_INVAL (cfg), PSL_E_STATE
 * (already serving), PSL_E_NOMEM (hbm_budget exceeds the device's free
 * memory), PSL_E_HIP. */
PSL_API psl_status psl_serve_start(psl_ctx *ctx, const psl_serve_cfg *cfg);

/* Queue a job; thread-safe and non-blocking. *ticket names it.
 * Errors: PSL_E_INVAL (bad job), PSL_E_FULL (its footprint exceeds the whole
 * budget), PSL_E_STATE (not serving). */
PSL_API psl_status psl_serve_submit(psl_ctx *ctx, const psl_job *job, uint64_t *ticket);

/* Thread-safe. PSL_OK: the job is finished, *out holds its result and the
 * ticket is retired. PSL_E_AGAIN: queued or running. PSL_E_STATE: unknown
 * (or already retired) ticket. */
PSL_API psl_status psl_serve_poll(psl_ctx *ctx, uint64_t ticket, psl_job_result *out);

/* Device bytes a job with this configuration counts against hbm_budget
 * (its walk slab, rounded up to its allocation class, plus an upper bound of
 * its share of the loop's scratch in any batch, at the default work-item
 * target). Needs no context or device. Errors: PSL_E_INVAL. */
PSL_API psl_status psl_serve_footprint(const psl_walk_cfg *cfg, uint64_t *bytes);

/* Thread-safe counters of the loop. */
PSL_API psl_status psl_serve_stats_read(psl_ctx *ctx, psl_serve_stats *out);

/* Stop the loop. drain != 0: finish every submitted job first; drain == 0:
 * cancel queued and running jobs. Results stay pollable until the next
 * psl_serve_start or psl_ctx_destroy. */
PSL_API psl_status psl_serve_stop(psl_ctx *ctx, int drain);

/* ------------------------------------------------------------ timing */

/* Per-kernel device time of psl_step_batch, measured with HIP events recorded
 * on the context's stream around each launch. */
typedef struct {
    double   eval_ms;        /* total time of the neighbourhood-evaluation kernel */
    uint64_t eval_launches;
    double   rest_ms;        /* total time of the rest of each step               */
    uint64_t steps;
    double   prep_ms;        /* split evaluation: its per-step preparation        */
    double   lin_ms;         /* split evaluation: the matrix-core linear sums     */
} psl_timing;

/* on != 0: start recording (counters reset); on == 0: stop. */
PSL_API psl_status psl_timing_enable(psl_ctx *ctx, int on);

/* Wait for the recorded work and report the totals since psl_timing_enable. */
PSL_API psl_status psl_timing_read(psl_ctx *ctx, psl_timing *out);

/* --------------------------------------------------------- autotuner */

/* Launch shape of the neighbourhood evaluation for a batch. */
typedef struct {
    int32_t waves;          /* wavefronts per block: 4, 8 or 16 (64 candidates each) */
    int32_t persistent;     /* 1: a fixed grid of blocks_per_cu x CUs takes work
                               items from per-XCD queues; 0: one block per item     */
    int32_t blocks_per_cu;  /* resident blocks per CU of the persistent grid: 1..3
                               (1..2 for 16 wavefronts, 1..6 for 4)                */
    int32_t eval_items;     /* work-item target kept with it (PSL_OPT_EVAL_ITEMS)   */
    double  eval_ms;        /* measured mean launch time of this shape              */
    double  default_ms;     /* measured mean launch time of the untuned default     */
} psl_tune_choice;

/* Time every candidate launch shape of the evaluation on these walks (their
 * state is not changed), then, in the fastest shape, the work-item targets
 * half, twice and four times PSL_OPT_EVAL_ITEMS; keep the fastest pair for
 * every later batch with the same key (log2 of the largest L, of the median
 * N_lmt and of the walk count, and whether the L differ by more than 4x),
 * and report it. Blocking.
 * Errors: PSL_E_INVAL, PSL_E_STATE, PSL_E_NOMEM, PSL_E_HIP. */
PSL_API psl_status psl_autotune(psl_ctx *ctx, const uint32_t *walk_ids, uint32_t n,
                                psl_tune_choice *out);

/* Write / read the context's tuned shapes as text (one "key waves persistent
 * blocks_per_cu eval_items" line each; a line without eval_items keeps the
 * context's value). Errors: PSL_E_INVAL (I/O or format). */
PSL_API psl_status psl_tune_save(psl_ctx *ctx, const char *path);
PSL_API psl_status psl_tune_load(psl_ctx *ctx, const char *path);

/* ----------------------------------------------------------- options */

/* PSL_OPT_NEAR_LIMIT: largest near-peak shift list (shifts k with |C_k|
 * within 8 of the pivot's PSL, the only ones that can set a neighbour's PSL)
 * for which the evaluation computes each neighbour's PSL from that list;
 * above it the PSL maximum is kept in the main loop. -1 (default): automatic,
 * min(4096, max(64, L/16)); 0 forces the in-loop maximum. Both give the same
 * results. Errors: PSL_E_INVAL for an unknown option or value. */
#define PSL_OPT_NEAR_LIMIT 1
/* PSL_OPT_EVAL_ITEMS: the number of work items (candidate tile x piece of
 * the shift range) an evaluation launch offers at least: a walk's shifts are
 * cut into pieces of about W / value shifts (at least 256), W being the
 * batch's total (candidate tile x shift) work. More items shorten the tail of
 * a launch over few long walks, at the cost of more partial sums to combine.
 * -1: the default, 4096; otherwise 1 .. 262144. It changes the grouping of
 * the FP64 F sums, so F only by rounding; PSL values are unaffected, and so
 * are the moves wherever the tolerance band decides them. Errors:
 * PSL_E_INVAL outside that range. */
#define PSL_OPT_EVAL_ITEMS 2
/* PSL_OPT_AMBIG_MARGIN: the relative margin m of the ambiguity flags
 * (PSL_CHOICE_AMBIGUOUS_ARGMIN, PSL_STEP_AMBIG_*), in units of 1e-15:
 * 0 .. 10^15 (m = 0 .. 1); -1 restores the default 500 (m = 5e-13, which
 * covers the FP64 rounding of this library's F, at most about 3e-14
 * relative, and of an exact summation). Only the flags change: the moves are
 * the band rule's whatever the margin. Errors: PSL_E_INVAL outside the range. */
#define PSL_OPT_AMBIG_MARGIN 3
/* PSL_OPT_SPLIT: the split evaluation (Eq. (5) expanded exactly in the +-1
 * neighbours of Section 3's one-element flip: the linear part of F_j as exact
 * integer sums on the matrix cores, the both-neighbour remainder on the
 * vector units) for walks of L >= 2048, in the steps that allow it (the
 * near-peak list holds the PSL and the quantization bound of the linear part
 * is below 1e-14 of every neighbour's F). 2 (default; -1 restores it): in
 * batches and evaluations whose walks of L >= 2048 hold at least 2^34
 * nominal updates (N_lmt x (L-1) summed), below which its fixed cost exceeds
 * what it saves; 1: in every batch and evaluation; 0: never (every step takes
 * the table evaluation). Moves and PSL are the same either way (F agrees to
 * about 1e-14 relative); errors: PSL_E_INVAL outside -1..2. */
#define PSL_OPT_SPLIT 4
/* PSL_OPT_TEST_FAIL_ADMIT: a test hook of the request loop. With n >= 1, the
 * n-th admission (counted per psl_serve_start, admissions that take at least
 * one job) fails with PSL_E_HIP before it launches anything, so the error path
 * can be exercised: its jobs finish with PSL_E_HIP, their slabs and slots are
 * released, and the loop goes on with the queue. 0 (default) turns it off.
 * Errors: PSL_E_INVAL for a negative value. */
#define PSL_OPT_TEST_FAIL_ADMIT 5
PSL_API psl_status psl_set_option(psl_ctx *ctx, int option, int64_t value);

/* --------------------------------------------------- trace, checkpoint */

/* One step of a walk as recorded by the trace ring. */
typedef struct {
    uint64_t t;             /* step number (0-based)                              */
    uint32_t start;         /* start of the limited neighbourhood                 */
    uint32_t k;             /* the move                                           */
    double   value_step;    /* F of the move                                      */
    int32_t  psl_k;         /* PSL of the move                                    */
    int32_t  psl_best;      /* best PSL after the step                            */
    uint32_t alpha;         /* exponent after the step                            */
    uint32_t flags;         /* PSL_STEP_* bits                                    */
} psl_trace_entry;

/* Record every later step of `walk` into a device ring of `capacity` entries
 * (0 stops recording and frees the ring). Errors: PSL_E_STATE, PSL_E_NOMEM. */
PSL_API psl_status psl_trace_enable(psl_ctx *ctx, uint32_t walk, uint32_t capacity);

/* Copy the most recent min(max_entries, recorded, capacity) entries, oldest
 * first, to host memory; *n_out receives the count. Waits for queued work.
 * Errors: PSL_E_STATE (unknown walk or no ring), PSL_E_HIP. */
PSL_API psl_status psl_trace_read(psl_ctx *ctx, uint32_t walk, psl_trace_entry *out,
                                  uint32_t max_entries, uint32_t *n_out);

/* Checkpoint restore: overwrite `walk` (same L) with a state read earlier by
 * psl_read_walk -- its scalars (exponent, v_local, psl_best, unimproved, t, q,
 * seed and control parameters) and its pivot, local_best and best bits (host,
 * ceil(L/64) words each). C, C of local_best and the pivot's F and PSL are
 * recomputed from the bits, so run N steps + read + restore + run M steps
 * equals N + M steps. Blocking. Errors: PSL_E_INVAL, PSL_E_STATE, PSL_E_HIP. */
PSL_API psl_status psl_restore_walk(psl_ctx *ctx, uint32_t walk, const psl_walk_state *state,
                                    const uint64_t *pivot_bits, const uint64_t *local_best_bits,
                                    const uint64_t *best_bits);

/* ----------------------------------------------------- introspection */

/* Candidate tiles (blocks of candidates) and k-splits the evaluation of one
 * walk of length L with n_lmt candidates uses when it is stepped in a batch
 * of n_walks such walks (1 <= n_walks <= 2^20), with the context's tuned
 * shapes and options when ctx is not NULL (for tests and bench). Errors:
 * PSL_E_INVAL. */
PSL_API psl_status psl_eval_shape(psl_ctx *ctx, uint32_t L, uint32_t n_lmt, uint32_t n_walks,
                          uint32_t *cand_tiles, uint32_t *k_splits);

/* Library version string. */
PSL_API const char *psl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PSL_H */
