// psl_internal.h -- host-side structures shared by the libpsl runtime and
// its serving loop (internal; not part of the C-ABI).
#pragma once

#include "psl.h"
#include "psl_device.h"
#include "psl_launch.h"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

namespace psl_rt {

using namespace psl;
using psl::EvalShape;
using psl::EvalQueues;

// ------------------------------------------------------------ arena

// First-fit allocator over a caller-provided device buffer. Offsets are
// 256-byte aligned; freed ranges merge with their neighbours.
class Arena {
public:
    void reset(char *base, size_t bytes)
    {
        base_ = base;
        free_.clear();
        if (base && bytes >= kAlign) free_[0] = bytes & ~(kAlign - 1);
    }
    bool active() const { return base_ != nullptr; }
    void *alloc(size_t bytes)
    {
        bytes = (bytes + kAlign - 1) & ~(kAlign - 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                used_[off] = bytes;
                return base_ + off;
            }
        }
        return nullptr;
    }
    void release(void *p)
    {
        size_t off = (size_t)((char *)p - base_);
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t len = u->second;
        used_.erase(u);
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + len == nx->first) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += len;
                return;
            }
        }
        free_[off] = len;
    }

private:
    static constexpr size_t kAlign = 256;
    char *base_ = nullptr;
    std::map<size_t, size_t> free_, used_;
};

// Host record of a walk slot.
struct WalkHost {
    bool active = false;
    uint32_t L = 0, nw = 0, n_lmt = 0, flip_lmt = 0;
    void *trace = nullptr;            // trace ring (hipMalloc), if enabled
    void *slab = nullptr;
    size_t slab_bytes = 0;
};

// A batch as laid out on the device; cached by its walk list.
struct BatchPlan {
    std::vector<uint32_t> ids;
    uint32_t max_L = 0, max_nw = 0;
    bool big_flips = false;           // some walk's Rand_flip exceeds the one-flip rebuild
    uint64_t pend_units = 0;          // work units of the pending-walk rebuild (all walks)
    uint32_t n_items = 0;
    EvalShape shape;                  // evaluation launch shape
    uint32_t comb_blocks = 1;         // combine blocks per walk (selection)
    uint32_t comb_group = 1;          // lanes per candidate in the combine
    EvalQueues *d_queues = nullptr;   // persistent evaluation: work queues
    BatchEntry *d_batch = nullptr;
    EvalItem *d_items = nullptr;
    bool carved = false;              // arrays carved from caller memory: not freed here
    hipGraph_t graph = nullptr;       // one captured step of this plan
    hipGraphExec_t gexec = nullptr;
    double *d_fpart = nullptr, *d_f = nullptr, *d_s0 = nullptr;
    uint32_t *d_mpart = nullptr, *d_m0 = nullptr, *d_near = nullptr;
    int32_t *d_p = nullptr;
    SelPart *d_red = nullptr;
    uint32_t *d_pend = nullptr;       // pending list: count, then batch positions
    uint32_t *d_done = nullptr;       // per batch position: combine blocks finished (0 between launches)
    uint32_t fixed_n = 0;             // plans of a fixed neighbourhood: its N_lmt (0: not fixed)
    uint32_t fixed_start = 0;         // ... and the start its batch entry holds
    uint32_t *d_seg = nullptr;        // segment map of the O(L) passes
    double *d_segtot = nullptr;       // per segment: chunk-sum total (suffix pass)
    uint32_t *d_segmax = nullptr;     // per segment: maximum |C_k|
    SegMap seg{};
    // split evaluation (walks with BatchEntry.lsplit > 0)
    bool split = false;               // some walk of the plan can take the split path
    int8_t *d_limbs = nullptr;
    double *d_dq = nullptr, *d_pre = nullptr, *d_lpart = nullptr;
    SplitState *d_ss = nullptr;
    EvalItem *d_litems = nullptr;     // linear items
    uint32_t n_litems = 0;
};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

constexpr size_t kPlanCache = 8;   // step batches whose layout (and graph) is kept
constexpr uint32_t kEvalItemsDefault = 4096;    // PSL_OPT_EVAL_ITEMS default
constexpr uint32_t kEvalItemsMax = 1u << 18;    // and its largest value
constexpr int64_t kAmbigMarginMax = 1000000000000000ll;  // PSL_OPT_AMBIG_MARGIN: 1.0 in units of 1e-15
constexpr uint32_t kSplitMinL = 2048;          // shortest walk the split evaluation takes
constexpr uint64_t kSplitMinWork = 1ull << 34; // fewest nominal updates of a launch that takes it
constexpr uint32_t kLinItemsTarget = 8192;     // linear items per launch the k-splits aim for
constexpr uint32_t kLinMinChunks = 256;         // fewest shift chunks per k-split of a linear item


struct Server;   // serving loop (psl_serve.hip)

}  // namespace psl_rt

struct psl_ctx {
    using Arena = psl_rt::Arena;
    using WalkHost = psl_rt::WalkHost;
    using BatchPlan = psl_rt::BatchPlan;
    using WalkDev = psl::WalkDev;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    Arena arena;
    std::vector<WalkHost> walks;
    std::vector<uint32_t> free_slots;
    WalkDev *d_walks = nullptr;
    uint32_t walk_cap = 0;
    double *d_T[PSL_ALPHA_MAX + 1] = {};
    uint32_t T_n = 0;                 // entries per power table
    std::vector<BatchPlan> plans;     // recent step batches, most recent last
    BatchPlan pure;                   // single-walk plan of psl_eval_neighbourhood (kept for the next call)
    psl::BatchEntry *d_one = nullptr; // psl_apply_flip's batch entry (allocated on first use)
    void *d_choice = nullptr;
    std::string err;
    int64_t near_limit = -1;          // PSL_OPT_NEAR_LIMIT
    uint32_t eval_items = psl_rt::kEvalItemsDefault;  // PSL_OPT_EVAL_ITEMS
    double amb_margin = psl::kAmbigMarginDefault;     // PSL_OPT_AMBIG_MARGIN (relative)
    int split_mode = 2;               // PSL_OPT_SPLIT: 2 by launch work, 1 wherever L allows, 0 never
    uint32_t test_fail_admit = 0;     // PSL_OPT_TEST_FAIL_ADMIT: serving admission n fails (0: never)
    void *noalloc_scratch = nullptr;  // this device's fixed scratch (psl_eval_neighbourhood_noalloc)
    std::string noalloc_err;          // why it is missing, if it is
    psl_rt::Server *server = nullptr; // serving loop, when started
    uint32_t n_cu = 256;              // compute units of the device
    std::map<uint32_t, psl::EvalShape> tuned;  // autotuner choices by tune_key
    std::map<uint32_t, uint32_t> tuned_items;  // autotuned work-item targets by tune_key
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev;       // 5 per recorded step (see timing_collect)
    double eval_ms = 0.0, rest_ms = 0.0, prep_ms = 0.0, lin_ms = 0.0;
    uint64_t eval_launches = 0, steps_timed = 0;
};

namespace psl_rt {

psl_status fail(psl_ctx *ctx, psl_status st, const char *fmt, ...);

#define HIP_TRY(ctx, expr)                                                              \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::psl_rt::fail((ctx), PSL_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

psl_status dev_alloc(psl_ctx *ctx, void **p, size_t bytes, bool from_arena);
void dev_free(psl_ctx *ctx, void *p, bool from_arena);
void plan_free(psl_ctx *ctx, BatchPlan &pl);
void plans_clear(psl_ctx *ctx);
psl_status ensure_tables(psl_ctx *ctx, uint32_t L);
Tables tables_of(const psl_ctx *ctx);
psl_status ensure_walk_cap(psl_ctx *ctx, uint32_t cap);
bool walk_ok(const psl_ctx *ctx, uint32_t id);
// Launch layout of a batch's evaluation: candidate tiles and k-splits per
// walk, and the work items in XCD-balanced order (see eval_layout).
struct EvalLayout {
    EvalShape shape;                  // launch shape the items are laid out for
    std::vector<uint32_t> tiles, ks;
    std::vector<EvalItem> items;      // flat: padded XCD ranges; persistent: queues
    EvalQueues queues{};              // persistent: queue ranges
    uint32_t comb_blocks = 1;         // combine blocks per walk (selection)
    uint32_t comb_group = 1;          // lanes per candidate in the combine
};
// Tuning key of a batch: (log2 of max L, log2 of the median N_lmt, log2 of
// the walk count, uneven flag).
uint32_t tune_key(const uint32_t *Ls, const uint32_t *n_lmt, uint32_t n);
// The evaluation shape for a batch: the tuned one for its key, else defaults.
EvalShape pick_shape(const psl_ctx *ctx, const uint32_t *Ls, const uint32_t *n_lmt, uint32_t n);
// min_items: the work items the launch should offer at least (the shifts of
// a walk split into pieces of about W / min_items, W the batch's total
// (candidate tile x shift) work).
void eval_layout(const uint32_t *Ls, const uint32_t *n_lmt, uint32_t n, const EvalShape &shape,
                 uint32_t min_items, EvalLayout &out);
void eval_shape_k(uint32_t L, uint32_t n_lmt, uint32_t K, uint32_t tile, uint32_t *tiles, uint32_t *ksplit);
uint32_t item_shifts_for(uint64_t W, uint32_t tile, uint32_t min_items);
uint32_t max_blocks_per_cu(int waves);
// Segment maps of the O(L) passes: every walk of length L; or off[0..n] =
// prefix sums of the walks' segment counts (the returned map's off is left
// null for the caller to point at the device copy).
SegMap seg_uniform(uint32_t nb, uint32_t L);
SegMap seg_prefix(const uint32_t *Ls, uint32_t n, uint32_t *off);
int eval_waves(const uint32_t *n_lmt, uint32_t n);
psl_status check_cfg(psl_ctx *ctx, const psl_walk_cfg *c);
// Device memory a plan's arrays come from instead of hipMalloc: a bump
// allocator over [base, base + cap) (256-byte aligned pieces), with the
// per-candidate F and PSL arrays given by the caller.
struct PlanMem {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    double *F = nullptr;
    int32_t *P = nullptr;
};
psl_status make_plan(psl_ctx *ctx, BatchPlan &pl, const uint32_t *ids, uint32_t n, uint32_t n_fixed,
                     uint32_t start_fixed, const EvalShape *force = nullptr, uint32_t force_items = 0,
                     PlanMem *mem = nullptr);
// The work-item target of a batch: the autotuned one for its key, else the
// context's PSL_OPT_EVAL_ITEMS; and the largest target any batch can get.
uint32_t items_for(const psl_ctx *ctx, const uint32_t *Ls, const uint32_t *n_lmt, uint32_t n);
uint32_t items_max(const psl_ctx *ctx);
uint32_t near_limit_for(const psl_ctx *ctx, uint32_t L);

// Slab layout of one walk of length L: the pivot between guard words, then
// local_best, best, C, C of local_best and the Rand_flip positions.
struct SlabLayout {
    size_t guard_bytes, pivot_bytes, bits_bytes, c_bytes, slab_bytes;
};
SlabLayout slab_layout(uint32_t L);
// Fills a WalkDev for cfg (seed already chosen) over a slab.
void fill_walk(WalkDev &w, const psl_walk_cfg &cfg, uint64_t seed, void *slab, const SlabLayout &lay);

// Stops the serving loop (if any) and releases it.
void serve_shutdown(psl_ctx *ctx);
// True while the serving loop owns the context.
bool serve_active(psl_ctx *ctx);

}  // namespace psl_rt
