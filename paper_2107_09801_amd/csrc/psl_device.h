// psl_device.h -- device-side layout of a walk and the kernel entry points.
//
// Internal to libpsl (not part of the C-ABI). One WalkDev per walk slot lives
// in device memory; kernels read and update it, the host copies it only at
// init and read-back.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psl {

constexpr double kTau = 1e-12;       // relative band of the best-neighbour and
                                     // improvement comparisons
constexpr int kEvalWavesMax = 16;    // wavefronts per evaluation block: 16, 8 or 4
constexpr int kEvalWaves = 8;        // the default below 256 x 1024 candidates per batch
constexpr int kEvalWavesSmall = 4;   // blocks for batches of small neighbourhoods
constexpr int kTileK = 256;          // shifts staged per LDS tile
constexpr int kChunks = kTileK / 32; // 32-shift windows per tile
constexpr int kPairs = kTileK / 2;   // shift pairs per tile
constexpr int kRowStride = 5;        // T(|C_k + 2m|), m = -2..2
constexpr int kNearCap = 4096;       // capacity of the near-peak shift list
constexpr uint32_t kFlipIncremental = 64;  // Rand_flip sizes rebuilt by one-flip updates

// Guard words (64-bit) before and after the pivot's bits: every bit window
// the evaluation reads (j +- k for j < L, k < L, plus one window) lies inside
// [-(nw+2)*64, (2*nw+2)*64), and the guards read as zero.
__host__ __device__ constexpr uint32_t guard_words(uint32_t nw) { return nw + 2; }

// Entries of the per-step chunk suffix arrays: one per 32-shift chunk of
// k = 1..L-1, plus a terminating zero.
__host__ __device__ constexpr uint32_t suffix_len(uint32_t L) { return (L - 1 + 31) / 32 + 1; }

struct WalkDev {
    // storage (slab)
    uint64_t *pivot;        // nw words
    uint64_t *local_best;   // nw words
    uint64_t *best;         // nw words (solution_best)
    int32_t *C;             // L entries, C[0] = L
    int32_t *C_lb;          // L entries: C of local_best
    uint32_t *flips;        // the positions of the last Rand_flip (<= flip_lmt)
    // control parameters
    uint64_t seed;
    uint32_t L, nw;
    uint32_t alpha1, alpha2;
    uint32_t n_lmt, ls_lmt, flip_lmt, switch_period;
    // state
    uint32_t alpha;
    uint32_t unimproved;
    uint64_t t;             // steps done
    uint64_t q;             // switches done
    double value_local;
    double F_pivot;
    int32_t psl_pivot;
    int32_t psl_best;
    // last step
    uint32_t start;
    uint32_t k;             // move (element index)
    uint32_t i_best;        // its scan index
    uint32_t j_psl;
    double value_step;
    double F_min;
    int32_t psl_k;
    int32_t psl_min;
    uint32_t flags;
    uint32_t pending;       // 1: C, F and PSL of the pivot must be rebuilt
    uint32_t n_flips;       // entries of flips[] for the pending rebuild
    uint32_t trace_cap;     // entries of the trace ring (0: no trace)
    struct TraceEntry *trace;   // ring, entry t % trace_cap for step t
};

// One step of the trace ring (layout of psl_trace_entry).
struct TraceEntry {
    uint64_t t;
    uint32_t start, k;
    double value_step;
    int32_t psl_k, psl_best;
    uint32_t alpha, flags;
};

struct Tables {
    const double *T[17];    // T[alpha][c] = c^alpha, left-to-right product
    uint32_t n;             // entries per table
    uint32_t pad;
};

// One walk of a batch, with its evaluation scratch (host-set per batch).
struct BatchEntry {
    double *Fpart;          // ksplit * n_lmt partial sums of T(|C'|)
    uint32_t *Mpart;        // ksplit * n_lmt partial maxima of hi32(T(|C'|))
    double *F;              // n_lmt: F per scan index
    int32_t *P;             // n_lmt: PSL per scan index
    double *S0;             // suffix_len(L): S0[x] = sum_{1+32x<=k'<L} T(|C_k'|), last = 0
    uint32_t *M0;           // suffix_len(L): max of hi32(T(|C_k'|)) over the same range
    uint32_t *near;         // 1 + kNearCap: count, then the near-peak shifts
    struct SelPart *red;    // combine blocks: per block minimum F and first minimum PSL
    uint32_t slot;          // walk slot
    uint32_t ksplit;        // k-splits of the evaluation
    uint32_t tiles;         // candidate tiles of the evaluation
    uint32_t n_lmt;         // candidates evaluated
    uint32_t start;         // start, when fixed by the caller
    uint32_t fixed;         // 1: start and n_lmt come from this entry
    uint32_t near_lim;      // largest near-peak list handled sparsely
    uint32_t lsplit;        // split path: k-splits of the linear items (0: no split path)
    // split path (psl_split.hip): this step's coefficients of the walk
    int8_t *limbs;          // [2][kLimbs][split_row(L)]: digits of B'_k (set 0) and B_k (set 1), shift k at k-1
    double *dq;             // [L][2]: D_k and B_k - B'_k
    double *pre;            // [3][L]: prefix sums over 1..k of A_k, A'_k, T(|C_k|); entry 0 is 0
    struct SplitState *ss;  // scale and path choice of this step
    double *lpart;          // [lsplit][L]: partial linear sums (in units of the scale), by element
};

// Split evaluation: T(|C_k + 2a + 2b|) = A + B(a + b) + D ab (both neighbours),
// T(|C_k + 2a|) = A' + B' a (one neighbour); the linear parts go to the
// matrix cores as exact integers (B' and B quantized to multiples of U, kLimbs
// signed byte digits), the rest to the VALU and to prefix sums.
constexpr int kLimbs = 8;
// Linear items: blocks of kLinBlockElems elements, kLinWaveElems per
// wavefront; a padding item has walk kLinNoWalk.
constexpr int kLinBlockElems = 4096;
// Digits per (set, limb) row: the 32-shift chunks of k = 1..L-1 and one more
// chunk of zeros (entries past L-1 are zero too).
__host__ __device__ constexpr uint32_t split_row(uint32_t L) { return 32u * ((L - 1 + 31) / 32 + 1); }
constexpr int kLinWaveElems = 1024;
constexpr uint32_t kLinNoWalk = 0xFFFFFFFFu;
struct SplitState {
    double U;               // the quantum, a power of two
    uint32_t use;           // 1: this step evaluates the walk on the split path
    uint32_t pad;
};

// Per combine block: the smallest F, and the smallest PSL with its first scan
// index, over the candidates the block combined.
struct SelPart {
    double f;
    int32_t p;
    uint32_t i;
};
constexpr uint32_t kCombMaxBlocks = 256;   // combine blocks per walk, at most

// Blocks of an O(L) pass over a batch: a walk's shifts k = 1..L-1 are cut
// into segments of 2^shift (256 .. 4096, chosen per batch so that the pass
// has a few thousand blocks); block i of the pass covers segment s of walk
// b. With off != nullptr, off[b] (b = 0..nb) are the prefix sums of the
// walks' segment counts (device memory); otherwise every walk has spw
// segments. total = the number of blocks.
constexpr uint32_t kSegShiftMin = 8, kSegShiftMax = 12;
__host__ __device__ constexpr uint32_t seg_count(uint32_t L, uint32_t shift)
{
    return (L - 1 + (1u << shift) - 1) >> shift;
}
struct SegMap {
    const uint32_t *off;
    uint32_t nb;
    uint32_t spw;
    uint32_t total;
    uint32_t shift;
    double *tot;            // per block: sum over its segment's chunks (or nullptr)
    uint32_t *tmax;         // per block: maximum |C_k| over its segment
};

constexpr uint32_t kNoItem = 0xFFFFFFFFu;  // padding work item (no work)

// Eval work item: walk position in the batch, candidate tile, k-split index.
struct EvalItem {
    uint32_t walk;
    uint32_t tile;
    uint32_t ks;
    uint32_t pad;
};

// XCDs of the MI355X (32 CUs and one L2 each); workgroup i of a launch runs
// on XCD i mod kXcds.
constexpr int kXcds = 8;

// Per-XCD work queues of the persistent evaluation: queue x holds the items
// base[x] .. base[x]+count[x]-1; next[x] is its cursor (reset per launch).
struct EvalQueues {
    uint32_t base[kXcds];
    uint32_t count[kXcds];
    uint32_t next[kXcds];
};

// Launch shape of the evaluation kernel.
struct EvalShape {
    int waves = kEvalWaves;     // wavefronts per block
    int persistent = 0;         // 1: fixed grid over the per-XCD queues
    uint32_t grid = 0;          // blocks of the persistent form
};

enum : uint32_t {
    STEP_IMPROVED = 1u,
    STEP_WORSE = 2u,
    STEP_SWITCHED = 4u,
    STEP_PSL_IMPROVED = 8u,
    STEP_AMBIG_ARGMIN = 16u,   // some neighbour's F lies within the margin of the band edge
    STEP_AMBIG_COMPARE = 32u,  // the move's F lies within the margin of a v_local band edge
};
constexpr uint32_t CHOICE_AMBIG_ARGMIN = 1u;
constexpr double kAmbigMarginDefault = 5e-13;   // relative ambiguity margin

}  // namespace psl
