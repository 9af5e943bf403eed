// psl_runtime.hip -- host runtime of libpsl: contexts, device memory, walks,
// batches and the C-ABI entry points declared in include/psl.h.
#include "psl_internal.h"

using namespace psl;
using namespace psl_rt;

// Fixed scratch of psl_eval_neighbourhood_noalloc: the evaluation plan's
// arrays of one walk (work items, k-split partials, chunk suffix arrays,
// near-peak list, combine minima, segment map, choice record), carved per
// call. Every device the library runs on holds one copy until the process
// ends, and every call on that device shares it. Host code reaches it only
// through the address hipGetSymbolAddress returns for the device (kept per
// device below); the array's own name is a host-side stand-in.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};   // device address of `scratch`, per device

// The device address of this device's scratch (the device is current),
// looked up once per device.
hipError_t scratch_address(int device, void **out)
{
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (!g_scratch_dev[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[device] = p;
    }
    *out = g_scratch_dev[device];
    return hipSuccess;
}
}  // namespace

namespace psl_rt {

psl_status fail(psl_ctx *ctx, psl_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return st;
}



psl_status dev_alloc(psl_ctx *ctx, void **p, size_t bytes, bool from_arena)
{
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    if (from_arena && ctx->arena.active()) {
        *p = ctx->arena.alloc(bytes);
        if (!*p) return fail(ctx, PSL_E_NOMEM, "arena exhausted (%zu bytes requested)", bytes);
        return PSL_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(ctx, PSL_E_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    return PSL_OK;
}

void dev_free(psl_ctx *ctx, void *p, bool from_arena)
{
    if (!p) return;
    if (from_arena && ctx->arena.active()) ctx->arena.release(p);
    else (void)hipFree(p);
}

void timing_drop(psl_ctx *ctx)
{
    for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
    ctx->ev.clear();
}

// Folds recorded events into the totals (the stream must be idle).
psl_status timing_collect(psl_ctx *ctx)
{
    // five events per step: evaluation start, after the split preparation,
    // after the evaluation kernel, after the linear sums, step end
    for (size_t i = 0; i + 4 < ctx->ev.size(); i += 5) {
        float a = 0.f, b = 0.f, c = 0.f, d = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&a, ctx->ev[i], ctx->ev[i + 1]));
        HIP_TRY(ctx, hipEventElapsedTime(&b, ctx->ev[i + 1], ctx->ev[i + 2]));
        HIP_TRY(ctx, hipEventElapsedTime(&c, ctx->ev[i + 2], ctx->ev[i + 3]));
        HIP_TRY(ctx, hipEventElapsedTime(&d, ctx->ev[i + 3], ctx->ev[i + 4]));
        ctx->prep_ms += a;
        ctx->eval_ms += b;
        ctx->lin_ms += c;
        ctx->rest_ms += d;
        ctx->eval_launches += 1;
        ctx->steps_timed += 1;
    }
    timing_drop(ctx);
    return PSL_OK;
}

psl_status timing_mark(psl_ctx *ctx)
{
    hipEvent_t e;
    HIP_TRY(ctx, hipEventCreate(&e));
    ctx->ev.push_back(e);
    HIP_TRY(ctx, hipEventRecord(e, ctx->stream));
    return PSL_OK;
}

void plan_free(psl_ctx *ctx, BatchPlan &pl)
{
    if (pl.gexec) (void)hipGraphExecDestroy(pl.gexec);
    if (pl.graph) (void)hipGraphDestroy(pl.graph);
    if (pl.carved) {
        pl = BatchPlan();
        return;
    }
    dev_free(ctx, pl.d_batch, false);
    dev_free(ctx, pl.d_items, false);
    dev_free(ctx, pl.d_fpart, false);
    dev_free(ctx, pl.d_mpart, false);
    dev_free(ctx, pl.d_f, false);
    dev_free(ctx, pl.d_p, false);
    dev_free(ctx, pl.d_s0, false);
    dev_free(ctx, pl.d_m0, false);
    dev_free(ctx, pl.d_red, false);
    dev_free(ctx, pl.d_pend, false);
    dev_free(ctx, pl.d_done, false);
    dev_free(ctx, pl.d_seg, false);
    dev_free(ctx, pl.d_segtot, false);
    dev_free(ctx, pl.d_segmax, false);
    dev_free(ctx, pl.d_near, false);
    dev_free(ctx, pl.d_queues, false);
    dev_free(ctx, pl.d_limbs, false);
    dev_free(ctx, pl.d_dq, false);
    dev_free(ctx, pl.d_pre, false);
    dev_free(ctx, pl.d_lpart, false);
    dev_free(ctx, pl.d_ss, false);
    dev_free(ctx, pl.d_litems, false);
    pl = BatchPlan();
}

void plans_clear(psl_ctx *ctx)
{
    for (auto &pl : ctx->plans) plan_free(ctx, pl);
    ctx->plans.clear();
    plan_free(ctx, ctx->pure);
}

// Power tables for every exponent, |c| up to L_max + 4.
psl_status ensure_tables(psl_ctx *ctx, uint32_t L)
{
    uint32_t need = L + 8;
    if (need <= ctx->T_n) return PSL_OK;
    uint32_t n = std::max<uint32_t>(need, 1024);
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    plans_clear(ctx);            // captured launches name the old tables
    for (uint32_t a = 1; a <= PSL_ALPHA_MAX; ++a) {
        dev_free(ctx, ctx->d_T[a], false);
        ctx->d_T[a] = nullptr;
    }
    ctx->T_n = 0;
    for (uint32_t a = 1; a <= PSL_ALPHA_MAX; ++a) {
        void *p;
        psl_status st = dev_alloc(ctx, &p, sizeof(double) * n, false);
        if (st) return st;
        ctx->d_T[a] = (double *)p;
        HIP_TRY(ctx, launch_power_table(ctx->d_T[a], n, a, ctx->stream));
    }
    ctx->T_n = n;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return PSL_OK;
}

Tables tables_of(const psl_ctx *ctx)
{
    Tables t;
    memset(&t, 0, sizeof t);
    for (uint32_t a = 1; a <= PSL_ALPHA_MAX; ++a) t.T[a] = ctx->d_T[a];
    t.n = ctx->T_n;
    return t;
}

psl_status ensure_walk_cap(psl_ctx *ctx, uint32_t cap)
{
    if (cap <= ctx->walk_cap) return PSL_OK;
    uint32_t ncap = std::max<uint32_t>(cap, std::max<uint32_t>(64, ctx->walk_cap * 2));
    void *p;
    psl_status st = dev_alloc(ctx, &p, sizeof(WalkDev) * ncap, false);
    if (st) return st;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    plans_clear(ctx);            // captured launches name the old walk array
    if (ctx->d_walks) {
        HIP_TRY(ctx, hipMemcpy(p, ctx->d_walks, sizeof(WalkDev) * ctx->walk_cap,
                               hipMemcpyDeviceToDevice));
        dev_free(ctx, ctx->d_walks, false);
    }
    ctx->d_walks = (WalkDev *)p;
    ctx->walk_cap = ncap;
    return PSL_OK;
}

bool walk_ok(const psl_ctx *ctx, uint32_t id)
{
    return id < ctx->walks.size() && ctx->walks[id].active;
}

// Evaluation shape of a batch. Candidates go in tiles of one block (64 lanes
// per wavefront; 4 wavefronts when most walks evaluate at most 256
// candidates, 16 for batches of at least 256 x 1024 candidates, else 8); the
// shifts of a walk split into pieces of K shifts (item_shifts_for), so a
// batch offers at least about 4096 work items (PSL_OPT_EVAL_ITEMS) and no
// item is much longer than the batch's average.
// Evaluation blocks resident per CU: the LDS of a block admits three; 16
// wavefronts per block are limited to two by the CU's wavefront slots.
// The largest segment (256 .. 4096 shifts) that still gives the pass about
// 2048 blocks.
static uint32_t seg_shift(uint64_t shifts)
{
    uint32_t sh = kSegShiftMax;
    while (sh > kSegShiftMin && (shifts >> sh) < 2048) --sh;
    return sh;
}

SegMap seg_uniform(uint32_t nb, uint32_t L)
{
    const uint32_t sh = seg_shift((uint64_t)nb * (L - 1));
    const uint32_t spw = seg_count(L, sh);
    return SegMap{nullptr, nb, spw, nb * spw, sh, nullptr, nullptr};
}

SegMap seg_prefix(const uint32_t *Ls, uint32_t n, uint32_t *off)
{
    uint64_t shifts = 0;
    for (uint32_t b = 0; b < n; ++b) shifts += Ls[b] - 1;
    const uint32_t sh = seg_shift(shifts);
    off[0] = 0;
    for (uint32_t b = 0; b < n; ++b) off[b + 1] = off[b] + seg_count(Ls[b], sh);
    return SegMap{nullptr, n, 0, off[n], sh, nullptr, nullptr};
}

// Resident evaluation blocks per CU: 16-wavefront blocks are held to two by
// their registers, 8-wavefront ones to three, 4-wavefront ones to six by
// their LDS.
uint32_t max_blocks_per_cu(int waves)
{
    return waves >= kEvalWavesMax ? 2u : waves == kEvalWavesSmall ? 6u : 3u;
}

int eval_waves(const uint32_t *nl, uint32_t n)
{
    uint32_t small = 0;
    uint64_t total = 0;
    for (uint32_t b = 0; b < n; ++b) {
        small += nl[b] <= 64u * kEvalWavesSmall;
        total += nl[b];
    }
    if (2 * small > n) return kEvalWavesSmall;
    // 16 wavefronts halve the per-candidate cost of building the LDS tables
    // once a batch has candidates for at least 256 such blocks
    return total >= 256ull * 64 * kEvalWavesMax ? kEvalWavesMax : kEvalWaves;
}

// Shifts per work item for W (candidate tile x shift) units of work: about
// W / min_items, but an item of more than 2^23 updates (K_big shifts of a
// tile) is cut down to K_big while the launch stays within max(65536,
// min_items) items. A launch over one or a few long walks otherwise has a
// few thousand items of several milliseconds each, whose different costs
// (both, one or no neighbour per shift) leave CUs idle at its end; batches
// of many walks keep one item per candidate tile.
uint32_t item_shifts_for(uint64_t W, uint32_t tile, uint32_t min_items)
{
    const uint64_t n_max = std::max<uint64_t>(65536, min_items);
    const uint64_t k_big = std::max<uint64_t>(kTileK, (1ull << 23) / tile);
    const uint64_t k = std::max<uint64_t>((W + n_max - 1) / n_max,
                                          std::min<uint64_t>(k_big, (W + min_items - 1) / min_items));
    return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(kTileK, k), UINT32_MAX);
}

static uint32_t item_shifts(const uint32_t *Ls, const uint32_t *nl, uint32_t n, uint32_t tile,
                            uint32_t min_items)
{
    uint64_t W = 0;
    for (uint32_t b = 0; b < n; ++b) W += (uint64_t)((nl[b] + tile - 1) / tile) * (Ls[b] - 1);
    return item_shifts_for(W, tile, min_items);
}

void eval_shape_k(uint32_t L, uint32_t n_lmt, uint32_t K, uint32_t tile, uint32_t *tiles, uint32_t *ksplit)
{
    *tiles = (n_lmt + tile - 1) / tile;
    const uint32_t nchunks = (L - 1 + 31) / 32;
    const uint32_t ks_max = std::max<uint32_t>(1, nchunks / (kTileK / 32));
    const uint32_t ks = (L - 1 + K - 1) / K;
    *ksplit = std::min(std::max<uint32_t>(ks, 1), ks_max);
}

uint32_t tune_key(const uint32_t *Ls, const uint32_t *nl, uint32_t n)
{
    uint32_t lmax = 0, lmin = UINT32_MAX;
    std::vector<uint32_t> v(nl, nl + n);
    for (uint32_t b = 0; b < n; ++b) {
        lmax = std::max(lmax, Ls[b]);
        lmin = std::min(lmin, Ls[b]);
    }
    std::nth_element(v.begin(), v.begin() + n / 2, v.end());
    auto lg = [](uint64_t x) { uint32_t r = 0; while (x > 1) { x >>= 1; ++r; } return r; };
    const uint32_t uneven = lmax > 4ull * lmin ? 1u : 0u;
    return lg(lmax) << 24 | lg(v[n / 2]) << 16 | lg(n) << 8 | uneven;
}

EvalShape pick_shape(const psl_ctx *ctx, const uint32_t *Ls, const uint32_t *nl, uint32_t n)
{
    auto it = ctx->tuned.find(tune_key(Ls, nl, n));
    if (it != ctx->tuned.end()) return it->second;
    EvalShape sh;
    sh.waves = eval_waves(nl, n);
    // launches of at least 2^38 nominal updates (about 10 ms): a fixed grid
    // over the per-XCD queues, which evens out items of different cost and
    // XCDs of different load; shorter launches pay more for the queues than
    // they gain and stay one block per item
    uint64_t updates = 0;
    for (uint32_t b = 0; b < n; ++b) updates += (uint64_t)nl[b] * (Ls[b] - 1);
    sh.persistent = updates >= (1ull << 38) ? 1 : 0;
    sh.grid = sh.persistent ? max_blocks_per_cu(sh.waves) * ctx->n_cu : 0;
    return sh;
}

void eval_layout(const uint32_t *Ls, const uint32_t *nl, uint32_t n, const EvalShape &shape,
                 uint32_t min_items, EvalLayout &out)
{
    out.shape = shape;
    out.tiles.assign(n, 0);
    out.ks.assign(n, 0);
    out.items.clear();
    const uint32_t tile = 64u * shape.waves;
    const uint32_t K = item_shifts(Ls, nl, n, tile, min_items);
    struct C { EvalItem it; double cost; };
    std::vector<C> all;
    double total = 0.0;
    for (uint32_t b = 0; b < n; ++b) {
        eval_shape_k(Ls[b], nl[b], K, tile, &out.tiles[b], &out.ks[b]);
        const uint32_t nchunks = (Ls[b] - 1 + 31) / 32;
        const uint32_t per = (nchunks + out.ks[b] - 1) / out.ks[b];
        for (uint32_t t = 0; t < out.tiles[b]; ++t) {
            const uint32_t cand = std::min<uint32_t>(tile, nl[b] - t * tile);
            for (uint32_t s = 0; s < out.ks[b]; ++s) {
                const uint32_t clo = s * per, chi = std::min(nchunks, clo + per);
                const double cost = (double)(chi > clo ? chi - clo : 0) * 32.0 * cand + 1.0;
                all.push_back(C{EvalItem{b, t, s, 0}, cost});
                total += cost;
            }
        }
    }
    // 8 contiguous segments of equal cost (one per XCD, so a walk's items
    // mostly share an L2), each in longest-first order. The one-block-per-
    // item form pads them to equal length (blocks map to XCDs round-robin);
    // the persistent form uses them as queues.
    std::vector<std::vector<C>> seg(8);
    double acc = 0.0;
    size_t x = 0;
    for (auto &c : all) {
        while (x < 7 && acc >= total * (double)(x + 1) / 8.0) ++x;
        seg[x].push_back(c);
        acc += c.cost;
    }
    size_t cmax = 0;
    for (auto &sg : seg) {
        std::stable_sort(sg.begin(), sg.end(), [](const C &a, const C &b) { return a.cost > b.cost; });
        cmax = std::max(cmax, sg.size());
    }
    // selection: a group of G lanes per candidate with about 16 splits per
    // lane, about 2048 partials per combine block, at most one block per
    // block-pass of candidates
    uint64_t work = 0, nmax = 0, ksmax = 1;
    for (uint32_t b = 0; b < n; ++b) {
        work = std::max<uint64_t>(work, (uint64_t)out.ks[b] * nl[b]);
        nmax = std::max<uint64_t>(nmax, nl[b]);
        ksmax = std::max<uint64_t>(ksmax, out.ks[b]);
    }
    uint32_t G = 1;
    while (G < 64 && (uint64_t)G * 16 < ksmax) G <<= 1;
    out.comb_group = G;
    const uint64_t cpb = 256 / G;
    // up to two blocks' worth of partials per walk: one block, which then
    // also makes the selection (no separate selection launch)
    out.comb_blocks = work <= 16384 ? 1u
                                    : (uint32_t)std::max<uint64_t>(
                                          1, std::min<uint64_t>({(work + 2047) / 2048, (nmax + cpb - 1) / cpb,
                                                                 (uint64_t)kCombMaxBlocks}));
    out.items.reserve(shape.persistent ? all.size() : 8 * cmax);
    for (int q = 0; q < 8; ++q) {
        auto &sg = seg[q];
        out.queues.base[q] = (uint32_t)out.items.size();
        out.queues.count[q] = (uint32_t)sg.size();
        out.queues.next[q] = 0;
        for (auto &c : sg) out.items.push_back(c.it);
        if (!shape.persistent)
            for (size_t k = sg.size(); k < cmax; ++k) out.items.push_back(EvalItem{kNoItem, 0, 0, 0});
    }
}

// Builds (or reuses) the device layout of a batch: entries, eval work items
// and scratch. n_fixed / start_fixed != UINT32_MAX: a pure single evaluation.
uint32_t items_for(const psl_ctx *ctx, const uint32_t *Ls, const uint32_t *nl, uint32_t n)
{
    auto it = ctx->tuned_items.find(tune_key(Ls, nl, n));
    return it != ctx->tuned_items.end() ? it->second : ctx->eval_items;
}

uint32_t items_max(const psl_ctx *ctx)
{
    uint32_t m = ctx->eval_items;
    for (const auto &kv : ctx->tuned_items) m = std::max(m, kv.second);
    return m;
}

psl_status make_plan(psl_ctx *ctx, BatchPlan &pl, const uint32_t *ids, uint32_t n, uint32_t n_fixed,
                     uint32_t start_fixed, const EvalShape *force, uint32_t force_items, PlanMem *mem)
{
    const bool fixed = n_fixed != UINT32_MAX;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    plan_free(ctx, pl);
    pl.ids.assign(ids, ids + n);
    pl.fixed_n = fixed ? n_fixed : 0;
    pl.fixed_start = fixed ? start_fixed : 0;
    std::vector<uint32_t> n_l(n), Ls(n);
    for (uint32_t b = 0; b < n; ++b) {
        const WalkHost &h = ctx->walks[ids[b]];
        n_l[b] = fixed ? n_fixed : h.n_lmt;
        Ls[b] = h.L;
        pl.big_flips |= h.flip_lmt > kFlipIncremental;
        pl.pend_units += pending_units(h.L);
        pl.max_L = std::max(pl.max_L, h.L);
        pl.max_nw = std::max(pl.max_nw, h.nw);
    }
    EvalLayout lay;
    const EvalShape shape = force ? *force : pick_shape(ctx, Ls.data(), n_l.data(), n);
    eval_layout(Ls.data(), n_l.data(), n, shape,
                force_items ? force_items : items_for(ctx, Ls.data(), n_l.data(), n), lay);
    const std::vector<uint32_t> &tiles = lay.tiles, &ks = lay.ks;
    std::vector<EvalItem> &items = lay.items;
    pl.shape = lay.shape;
    pl.comb_blocks = lay.comb_blocks;
    pl.comb_group = lay.comb_group;
    size_t n_part = 0, n_cand = 0, n_suf = 0;
    for (uint32_t b = 0; b < n; ++b) {
        n_part += (size_t)ks[b] * n_l[b];
        n_cand += n_l[b];
        n_suf += suffix_len(Ls[b]);
    }
    const uint64_t n_items = items.size();
    if (n_items >= (1ull << 31)) return fail(ctx, PSL_E_INVAL, "batch too large (%llu work items)",
                                             (unsigned long long)n_items);
    if (mem) {
        // every array of the plan comes from mem; F and PSL are the caller's
        pl.carved = true;
        if (n != 1 || !mem->F || !mem->P) return fail(ctx, PSL_E_INVAL, "carved plans are single-walk");
    }
    auto get = [&](void **q, size_t bytes) -> psl_status {
        if (!mem) return dev_alloc(ctx, q, bytes, false);
        const size_t need = align_up(std::max<size_t>(bytes, 1), 256);
        if (need > mem->cap - mem->used)
            return fail(ctx, PSL_E_NOMEM, "the evaluation needs more than the %zu bytes of fixed scratch",
                        mem->cap);
        *q = mem->base + mem->used;
        mem->used += need;
        return PSL_OK;
    };
    void *p;
    psl_status st;
    if ((st = get(&p, sizeof(double) * n_part))) return st;
    pl.d_fpart = (double *)p;
    if ((st = get(&p, sizeof(uint32_t) * n_part))) return st;
    pl.d_mpart = (uint32_t *)p;
    if (mem) {
        pl.d_f = mem->F;
        pl.d_p = mem->P;
    } else {
        if ((st = get(&p, sizeof(double) * n_cand))) return st;
        pl.d_f = (double *)p;
        if ((st = get(&p, sizeof(int32_t) * n_cand))) return st;
        pl.d_p = (int32_t *)p;
    }
    if ((st = get(&p, sizeof(double) * n_suf))) return st;
    pl.d_s0 = (double *)p;
    if ((st = get(&p, sizeof(uint32_t) * n_suf))) return st;
    pl.d_m0 = (uint32_t *)p;
    if ((st = get(&p, sizeof(uint32_t) * (kNearCap + 1) * n))) return st;
    pl.d_near = (uint32_t *)p;
    if ((st = get(&p, sizeof(SelPart) * pl.comb_blocks * n))) return st;
    pl.d_red = (SelPart *)p;
    if ((st = get(&p, sizeof(uint32_t) * (n + 1)))) return st;
    pl.d_pend = (uint32_t *)p;
    if ((st = get(&p, sizeof(uint32_t) * n))) return st;
    pl.d_done = (uint32_t *)p;
    {
        std::vector<uint32_t> off(n + 1);
        pl.seg = seg_prefix(Ls.data(), n, off.data());
        if ((st = get(&p, sizeof(uint32_t) * (n + 1)))) return st;
        pl.d_seg = (uint32_t *)p;
        pl.seg.off = pl.d_seg;
        HIP_TRY(ctx, hipMemcpy(pl.d_seg, off.data(), sizeof(uint32_t) * (n + 1), hipMemcpyHostToDevice));
        if ((st = get(&p, sizeof(double) * pl.seg.total))) return st;
        pl.d_segtot = (double *)p;
        if ((st = get(&p, sizeof(uint32_t) * pl.seg.total))) return st;
        pl.d_segmax = (uint32_t *)p;
        pl.seg.tot = pl.d_segtot;
        pl.seg.tmax = pl.d_segmax;
    }
    // split evaluation: per walk of at least kSplitMinL elements (not for
    // plans carved from fixed scratch, nor for launches with less work than
    // kSplitMinWork nominal updates, where its fixed cost exceeds what it
    // saves): its coefficient arrays, linear partials and linear items (walk,
    // kLinBlockElems-element block, k-split). Workgroup i runs on XCD i mod 8:
    // each walk's items (cost: the chunks of its k-split) form one piece, or
    // several of consecutive items when the walk holds more than 1/16 of the
    // launch's cost; the pieces are dealt to 8 queues (costliest first, each
    // to the least loaded queue) and the launch order interleaves the queues,
    // so XCD x takes queue x. A batch of many walks keeps each walk's items
    // (and its digits in L2) on one XCD, and one long walk spreads over all
    // eight; short queues are padded with kLinNoWalk items.
    std::vector<uint32_t> lsp(n, 0);
    std::vector<EvalItem> litems;
    size_t n_limb = 0, n_dq = 0, n_pre = 0, n_lp = 0;
    uint64_t split_work = 0;
    for (uint32_t b = 0; b < n; ++b)
        if (Ls[b] >= kSplitMinL) split_work += (uint64_t)n_l[b] * (Ls[b] - 1);
    if (!mem && (ctx->split_mode == 1 || (ctx->split_mode == 2 && split_work >= kSplitMinWork))) {
        uint64_t blocks = 0;
        std::vector<uint32_t> nq(n, 0);
        for (uint32_t b = 0; b < n; ++b) {
            if (Ls[b] < kSplitMinL) continue;
            const uint32_t nblk = (Ls[b] + kLinBlockElems - 1) / kLinBlockElems;
            nq[b] = std::min<uint32_t>(nblk, (n_l[b] + kLinBlockElems - 1) / kLinBlockElems + 1);
            blocks += nq[b];
        }
        struct Piece {
            uint32_t b, first, count;   // items first .. first+count-1 of walk b (q-major, k-split minor)
            uint64_t cost;
        };
        std::vector<Piece> pieces;
        std::vector<uint64_t> item_cost(n, 0);
        uint64_t total = 0;
        for (uint32_t b = 0; b < n; ++b) {
            if (!nq[b]) continue;
            const uint32_t nchunks = (Ls[b] - 1 + 31) / 32;
            const uint64_t want = (kLinItemsTarget + blocks - 1) / std::max<uint64_t>(blocks, 1);
            lsp[b] = (uint32_t)std::max<uint64_t>(
                1, std::min<uint64_t>(want, std::max<uint32_t>(1, nchunks / kLinMinChunks)));
            item_cost[b] = (nchunks + lsp[b] - 1) / lsp[b];
            total += item_cost[b] * nq[b] * lsp[b];
            n_limb += 2 * (size_t)kLimbs * split_row(Ls[b]);
            n_dq += 2 * (size_t)Ls[b];
            n_pre += 3 * (size_t)Ls[b];
            n_lp += (size_t)lsp[b] * Ls[b];
        }
        const uint64_t cap = std::max<uint64_t>(1, total / 16);
        for (uint32_t b = 0; b < n; ++b) {
            if (!nq[b]) continue;
            const uint32_t items = nq[b] * lsp[b];
            const uint64_t cost = item_cost[b] * items;
            const uint32_t np = (uint32_t)std::min<uint64_t>(items, (cost + cap - 1) / cap);
            for (uint32_t p = 0; p < np; ++p) {
                const uint32_t lo = (uint32_t)((uint64_t)items * p / np), hi = (uint32_t)((uint64_t)items * (p + 1) / np);
                pieces.push_back(Piece{b, lo, hi - lo, item_cost[b] * (hi - lo)});
            }
        }
        std::stable_sort(pieces.begin(), pieces.end(), [](const Piece &a, const Piece &c) { return a.cost > c.cost; });
        std::vector<EvalItem> xq[kXcds];
        uint64_t load[kXcds] = {};
        for (const Piece &pc : pieces) {
            const int x = (int)(std::min_element(load, load + kXcds) - load);
            for (uint32_t i = pc.first; i < pc.first + pc.count; ++i)
                xq[x].push_back(EvalItem{pc.b, i / lsp[pc.b], i % lsp[pc.b], 0});
            load[x] += pc.cost;
        }
        size_t rounds = 0;
        for (int x = 0; x < kXcds; ++x) rounds = std::max(rounds, xq[x].size());
        for (size_t r = 0; r < rounds; ++r)
            for (int x = 0; x < kXcds; ++x)
                litems.push_back(r < xq[x].size() ? xq[x][r] : EvalItem{kLinNoWalk, 0, 0, 0});
    }
    pl.split = !litems.empty();
    if (pl.split) {
        if ((st = get(&p, n_limb))) return st;
        pl.d_limbs = (int8_t *)p;
        if ((st = get(&p, sizeof(double) * n_dq))) return st;
        pl.d_dq = (double *)p;
        if ((st = get(&p, sizeof(double) * n_pre))) return st;
        pl.d_pre = (double *)p;
        if ((st = get(&p, sizeof(double) * n_lp))) return st;
        pl.d_lpart = (double *)p;
        if ((st = get(&p, sizeof(SplitState) * n))) return st;
        pl.d_ss = (SplitState *)p;
        if ((st = get(&p, sizeof(EvalItem) * litems.size()))) return st;
        pl.d_litems = (EvalItem *)p;
        pl.n_litems = (uint32_t)litems.size();
        HIP_TRY(ctx, hipMemcpy(pl.d_litems, litems.data(), sizeof(EvalItem) * litems.size(),
                               hipMemcpyHostToDevice));
    }
    std::vector<BatchEntry> be(n);
    size_t op = 0, oc = 0, os = 0;
    size_t o_limb = 0, o_dq = 0, o_pre = 0, o_lp = 0;
    for (uint32_t b = 0; b < n; ++b) {
        BatchEntry &e = be[b];
        memset(&e, 0, sizeof e);
        e.Fpart = pl.d_fpart + op;
        e.Mpart = pl.d_mpart + op;
        e.F = pl.d_f + oc;
        e.P = pl.d_p + oc;
        e.S0 = pl.d_s0 + os;
        e.M0 = pl.d_m0 + os;
        e.near = pl.d_near + (size_t)(kNearCap + 1) * b;
        e.red = pl.d_red + (size_t)pl.comb_blocks * b;
        os += suffix_len(ctx->walks[ids[b]].L);
        e.slot = ids[b];
        e.ksplit = ks[b];
        e.tiles = tiles[b];
        e.n_lmt = n_l[b];
        e.start = fixed ? start_fixed : 0;
        e.near_lim = near_limit_for(ctx, ctx->walks[ids[b]].L);
        e.fixed = fixed ? 1 : 0;
        if (lsp[b]) {
            const size_t K = split_row(Ls[b]);
            e.lsplit = lsp[b];
            e.limbs = pl.d_limbs + o_limb;
            e.dq = pl.d_dq + o_dq;
            e.pre = pl.d_pre + o_pre;
            e.lpart = pl.d_lpart + o_lp;
            e.ss = pl.d_ss + b;
            o_limb += 2 * (size_t)kLimbs * K;
            o_dq += 2 * (size_t)Ls[b];
            o_pre += 3 * (size_t)Ls[b];
            o_lp += (size_t)lsp[b] * Ls[b];
        }
        op += (size_t)ks[b] * n_l[b];
        oc += n_l[b];
    }
    if ((st = get(&p, sizeof(BatchEntry) * n))) return st;
    pl.d_batch = (BatchEntry *)p;
    if ((st = get(&p, sizeof(EvalItem) * std::max<size_t>(items.size(), 1)))) return st;
    pl.d_items = (EvalItem *)p;
    if ((st = get(&p, sizeof(EvalQueues)))) return st;
    pl.d_queues = (EvalQueues *)p;
    HIP_TRY(ctx, hipMemcpy(pl.d_queues, &lay.queues, sizeof(EvalQueues), hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(pl.d_batch, be.data(), sizeof(BatchEntry) * n, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(pl.d_items, items.data(), sizeof(EvalItem) * items.size(),
                           hipMemcpyHostToDevice));
    HIP_TRY(ctx, launch_near_reset(pl.d_batch, n, pl.d_pend, pl.d_done, ctx->stream));
    pl.n_items = (uint32_t)items.size();
    return PSL_OK;
}

SlabLayout slab_layout(uint32_t L)
{
    const uint32_t nw = (L + 63) / 64;
    SlabLayout s;
    s.bits_bytes = align_up(sizeof(uint64_t) * nw, 256);
    s.guard_bytes = sizeof(uint64_t) * guard_words(nw);
    s.pivot_bytes = align_up(2 * s.guard_bytes + sizeof(uint64_t) * nw, 256);
    s.c_bytes = align_up(sizeof(int32_t) * L, 256);
    s.slab_bytes = s.pivot_bytes + 2 * s.bits_bytes + 2 * s.c_bytes + align_up(4 * PSL_FLIP_LMT_MAX, 256);
    return s;
}

void fill_walk(WalkDev &w, const psl_walk_cfg &cfg, uint64_t seed, void *slab, const SlabLayout &lay)
{
    memset(&w, 0, sizeof w);
    char *base = (char *)slab;
    w.pivot = (uint64_t *)(base + lay.guard_bytes);
    w.local_best = (uint64_t *)(base + lay.pivot_bytes);
    w.best = (uint64_t *)(base + lay.pivot_bytes + lay.bits_bytes);
    w.C = (int32_t *)(base + lay.pivot_bytes + 2 * lay.bits_bytes);
    w.C_lb = (int32_t *)(base + lay.pivot_bytes + 2 * lay.bits_bytes + lay.c_bytes);
    w.flips = (uint32_t *)(base + lay.pivot_bytes + 2 * lay.bits_bytes + 2 * lay.c_bytes);
    w.seed = seed;
    w.L = cfg.L;
    w.nw = (cfg.L + 63) / 64;
    w.alpha1 = cfg.alpha1;
    w.alpha2 = cfg.alpha2;
    w.alpha = cfg.alpha1;
    w.n_lmt = cfg.n_lmt ? cfg.n_lmt : cfg.L;
    w.ls_lmt = cfg.ls_lmt;
    w.flip_lmt = cfg.flip_lmt;
    w.switch_period = cfg.switch_period;
}

uint32_t near_limit_for(const psl_ctx *ctx, uint32_t L)
{
    const uint32_t autol = std::min<uint32_t>(kNearCap, std::max<uint32_t>(64, L / 16));
    return ctx->near_limit < 0 ? autol : (uint32_t)std::min<int64_t>(ctx->near_limit, kNearCap);
}

psl_status check_cfg(psl_ctx *ctx, const psl_walk_cfg *c)
{
    if (!c) return fail(ctx, PSL_E_INVAL, "cfg is NULL");
    if (c->L < 2 || c->L > PSL_L_MAX) return fail(ctx, PSL_E_INVAL, "L=%u out of [2, %u]", c->L, PSL_L_MAX);
    if (c->alpha1 < 1 || c->alpha1 > PSL_ALPHA_MAX || c->alpha2 < 1 || c->alpha2 > PSL_ALPHA_MAX)
        return fail(ctx, PSL_E_INVAL, "alpha out of [1, %u]", PSL_ALPHA_MAX);
    if (c->n_lmt > c->L) return fail(ctx, PSL_E_INVAL, "n_lmt=%u > L=%u", c->n_lmt, c->L);
    if (c->flip_lmt > c->L || c->flip_lmt > PSL_FLIP_LMT_MAX)
        return fail(ctx, PSL_E_INVAL, "flip_lmt=%u out of range", c->flip_lmt);
    if (c->reserved != 0) return fail(ctx, PSL_E_INVAL, "reserved must be 0");
    return PSL_OK;
}

// The launches of one iteration of Algorithm 1 for every walk of a plan.
psl_status launch_step(psl_ctx *ctx, const BatchPlan &pl, const Tables &tabs, uint32_t n, bool timed)
{
    psl_status st;
    HIP_TRY(ctx, launch_suffix(ctx->d_walks, pl.d_batch, n, pl.max_L, tabs, 0, &pl.seg, pl.d_pend,
                               pl.shape.waves >= kEvalWavesMax, ctx->stream));
    if (timed && (st = timing_mark(ctx))) return st;
    if (pl.split) HIP_TRY(ctx, launch_split_prep(ctx->d_walks, pl.d_batch, n, tabs, pl.seg, ctx->stream));
    if (timed && (st = timing_mark(ctx))) return st;
    HIP_TRY(ctx, launch_eval(ctx->d_walks, pl.d_batch, pl.d_items, pl.n_items, tabs, pl.shape, pl.d_queues,
                             ctx->stream));
    if (timed && (st = timing_mark(ctx))) return st;
    if (pl.split) HIP_TRY(ctx, launch_lin(ctx->d_walks, pl.d_batch, pl.d_litems, pl.n_litems, ctx->stream));
    if (timed && (st = timing_mark(ctx))) return st;
    HIP_TRY(ctx, launch_select(ctx->d_walks, pl.d_batch, n, pl.comb_blocks, pl.comb_group, tabs, 0, nullptr,
                               pl.d_pend, pl.d_done, ctx->amb_margin, ctx->stream));
    HIP_TRY(ctx, launch_apply(ctx->d_walks, pl.d_batch, pl.seg, -1, ctx->stream));
    if (pl.big_flips) HIP_TRY(ctx, launch_corr(ctx->d_walks, pl.d_batch, n, pl.max_L, 1, ctx->stream));
    HIP_TRY(ctx, launch_pending(ctx->d_walks, pl.d_batch, n, pl.pend_units, tabs, pl.d_pend, ctx->stream));
    if (timed && (st = timing_mark(ctx))) return st;
    return PSL_OK;
}

// Captures one step of the plan into a graph (every per-step quantity lives
// in device memory, so one capture serves every later step).
psl_status capture_step(psl_ctx *ctx, BatchPlan &pl, const Tables &tabs, uint32_t n)
{
    HIP_TRY(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    psl_status st = launch_step(ctx, pl, tabs, n, false);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->stream, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(ctx, PSL_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&pl.gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        pl.gexec = nullptr;
        return fail(ctx, PSL_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    pl.graph = g;
    return PSL_OK;
}

// The context's one-walk batch entry (psl_apply_flip, psl_restore_walk),
// allocated on first use and kept until the context is destroyed.
psl_status one_entry(psl_ctx *ctx)
{
    if (ctx->d_one) return PSL_OK;
    void *p;
    const psl_status st = dev_alloc(ctx, &p, sizeof(BatchEntry), false);
    if (st) return st;
    ctx->d_one = (BatchEntry *)p;
    return PSL_OK;
}

}  // namespace psl_rt

// ================================================================= C-ABI

extern "C" {

const char *psl_version(void) { return "libpsl 0.1 (gfx950)"; }

psl_status psl_ctx_create(int device, void *hip_stream, void *arena, size_t arena_bytes, psl_ctx **out)
{
    if (!out) return PSL_E_INVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return PSL_E_INVAL;
    }
    psl_ctx *ctx = new psl_ctx();
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return PSL_E_HIP;
    }
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return PSL_E_HIP;
        }
        ctx->own_stream = true;
    }
    if (arena) ctx->arena.reset((char *)arena, arena_bytes);
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
            ctx->n_cu = (uint32_t)cus;
        (void)hipGetLastError();
    }
    {
        // the fixed scratch of psl_eval_neighbourhood_noalloc on this device;
        // without it that call fails and every other call works
        const hipError_t e = scratch_address(device, &ctx->noalloc_scratch);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            ctx->noalloc_scratch = nullptr;
            ctx->noalloc_err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
        }
    }
    if (hipMalloc(&ctx->d_choice, 256) != hipSuccess) {
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
        delete ctx;
        return PSL_E_HIP;
    }
    *out = ctx;
    return PSL_OK;
}

void psl_ctx_destroy(psl_ctx *ctx)
{
    if (!ctx) return;
    serve_shutdown(ctx);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &h : ctx->walks) {
        if (h.active) dev_free(ctx, h.slab, true);
        dev_free(ctx, h.trace, false);
    }
    plans_clear(ctx);
    for (uint32_t a = 1; a <= PSL_ALPHA_MAX; ++a) dev_free(ctx, ctx->d_T[a], false);
    dev_free(ctx, ctx->d_walks, false);
    dev_free(ctx, ctx->d_choice, false);
    dev_free(ctx, ctx->d_one, false);
    timing_drop(ctx);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char *psl_last_error(const psl_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

psl_status psl_sync(psl_ctx *ctx)
{
    if (!ctx) return PSL_E_INVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return PSL_OK;
}

psl_status psl_init_walks(psl_ctx *ctx, const psl_walk_cfg *cfg, uint32_t n,
                          const uint64_t *const *init_bits, uint32_t *walk_ids_out)
{
    if (!ctx) return PSL_E_INVAL;
    if (serve_active(ctx)) return fail(ctx, PSL_E_STATE, "the context is serving");
    psl_status st = check_cfg(ctx, cfg);
    if (st) return st;
    if (n == 0) return PSL_OK;
    if (!walk_ids_out) return fail(ctx, PSL_E_INVAL, "walk_ids_out is NULL");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if ((st = ensure_tables(ctx, cfg->L))) return st;

    const uint32_t L = cfg->L, nw = (L + 63) / 64;
    const SlabLayout lay = slab_layout(L);
    const size_t slab_bytes = lay.slab_bytes;

    // slots
    std::vector<uint32_t> ids(n);
    for (uint32_t b = 0; b < n; ++b) {
        if (!ctx->free_slots.empty()) {
            ids[b] = ctx->free_slots.back();
            ctx->free_slots.pop_back();
        } else {
            ids[b] = (uint32_t)ctx->walks.size();
            ctx->walks.push_back(WalkHost());
        }
    }
    auto rollback = [&](uint32_t upto) {
        for (uint32_t b = 0; b < n; ++b) {
            WalkHost &h = ctx->walks[ids[b]];
            if (b < upto && h.slab) dev_free(ctx, h.slab, true);
            h = WalkHost();
            ctx->free_slots.push_back(ids[b]);
        }
    };
    if ((st = ensure_walk_cap(ctx, (uint32_t)ctx->walks.size()))) {
        rollback(0);
        return st;
    }
    std::vector<WalkDev> wd(n);
    std::vector<uint32_t> want(n);
    for (uint32_t b = 0; b < n; ++b) {
        void *slab;
        if ((st = dev_alloc(ctx, &slab, slab_bytes, true))) {
            rollback(b);
            return st;
        }
        WalkHost &h = ctx->walks[ids[b]];
        h.active = true;
        h.L = L;
        h.nw = nw;
        h.n_lmt = cfg->n_lmt ? cfg->n_lmt : L;
        h.flip_lmt = cfg->flip_lmt;
        h.slab = slab;
        h.slab_bytes = slab_bytes;
        WalkDev &w = wd[b];
        // the pivot sits between zeroed guard words (see guard_words)
        HIP_TRY(ctx, hipMemsetAsync(slab, 0, slab_bytes, ctx->stream));
        fill_walk(w, *cfg, cfg->seed + b, slab, lay);
        const uint64_t *given = init_bits ? init_bits[b] : nullptr;
        want[b] = given ? 0u : 1u;
        if (given) {
            uint64_t last = given[nw - 1];
            if ((L & 63u) && (last >> (L & 63u))) {
                rollback(b + 1);
                return fail(ctx, PSL_E_INVAL, "init_bits[%u] has bits set at or beyond L", b);
            }
            HIP_TRY(ctx, hipMemcpyAsync(w.pivot, given, sizeof(uint64_t) * nw,
                                        hipMemcpyHostToDevice, ctx->stream));
        }
        HIP_TRY(ctx, hipMemcpyAsync(ctx->d_walks + ids[b], &w, sizeof(WalkDev),
                                    hipMemcpyHostToDevice, ctx->stream));
    }
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    // init plan: entries and the chunk arrays of the fitness pass, on a
    // temporary plan
    BatchPlan tmp;
    {
        void *p;
        if ((st = dev_alloc(ctx, &p, sizeof(BatchEntry) * n, false))) return st;
        tmp.d_batch = (BatchEntry *)p;
        const size_t ns = suffix_len(L);
        if ((st = dev_alloc(ctx, &p, sizeof(double) * ns * n, false))) {
            plan_free(ctx, tmp);
            return st;
        }
        tmp.d_s0 = (double *)p;
        if ((st = dev_alloc(ctx, &p, sizeof(uint32_t) * ns * n, false))) {
            plan_free(ctx, tmp);
            return st;
        }
        tmp.d_m0 = (uint32_t *)p;
        std::vector<BatchEntry> be(n);
        for (uint32_t b = 0; b < n; ++b) {
            memset(&be[b], 0, sizeof(BatchEntry));
            be[b].slot = ids[b];
            be[b].S0 = tmp.d_s0 + ns * b;
            be[b].M0 = tmp.d_m0 + ns * b;
        }
        void *dw;
        if ((st = dev_alloc(ctx, &dw, sizeof(uint32_t) * n, false))) {
            plan_free(ctx, tmp);
            return st;
        }
        HIP_TRY(ctx, hipMemcpy(tmp.d_batch, be.data(), sizeof(BatchEntry) * n, hipMemcpyHostToDevice));
        HIP_TRY(ctx, hipMemcpy(dw, want.data(), sizeof(uint32_t) * n, hipMemcpyHostToDevice));
        const Tables tabs = tables_of(ctx);
        hipError_t e = launch_init_bits(ctx->d_walks, tmp.d_batch, (const uint32_t *)dw, n, nw, ctx->stream);
        if (e == hipSuccess) e = launch_corr(ctx->d_walks, tmp.d_batch, n, L, 0, ctx->stream);
        const SegMap sm = seg_uniform(n, L);
        if (e == hipSuccess) e = launch_suffix(ctx->d_walks, tmp.d_batch, n, L, tabs, 2, &sm, nullptr, 0, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        dev_free(ctx, dw, false);
        plan_free(ctx, tmp);
        if (e != hipSuccess) return fail(ctx, PSL_E_HIP, "walk init: %s", hipGetErrorString(e));
    }
    memcpy(walk_ids_out, ids.data(), sizeof(uint32_t) * n);
    return PSL_OK;
}

psl_status psl_free_walks(psl_ctx *ctx, const uint32_t *walk_ids, uint32_t n)
{
    if (!ctx || (n && !walk_ids)) return PSL_E_INVAL;
    if (serve_active(ctx)) return fail(ctx, PSL_E_STATE, "the context is serving");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    psl_status st = PSL_OK;
    for (uint32_t b = 0; b < n; ++b) {
        uint32_t id = walk_ids[b];
        if (!walk_ok(ctx, id)) {
            st = fail(ctx, PSL_E_STATE, "unknown walk %u", id);
            continue;
        }
        WalkHost &h = ctx->walks[id];
        dev_free(ctx, h.slab, true);
        dev_free(ctx, h.trace, false);
        h = WalkHost();
        ctx->free_slots.push_back(id);
    }
    plans_clear(ctx);            // cached layouts may name freed walks
    return st;
}

psl_status psl_eval_neighbourhood(psl_ctx *ctx, uint32_t walk, uint32_t start, uint32_t n_lmt,
                                  double *F_dev, int32_t *psl_dev, psl_choice *out)
{
    if (!ctx) return PSL_E_INVAL;
    if (serve_active(ctx)) return fail(ctx, PSL_E_STATE, "the context is serving");
    if (!walk_ok(ctx, walk)) return fail(ctx, PSL_E_STATE, "unknown walk %u", walk);
    const WalkHost &h = ctx->walks[walk];
    if (n_lmt < 1 || n_lmt > h.L || start >= h.L)
        return fail(ctx, PSL_E_INVAL, "start=%u n_lmt=%u for L=%u", start, n_lmt, h.L);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    // The plan of the previous call serves again when it was made for the
    // same walk and N_lmt (freeing walks or changing options drops it): its
    // layout does not depend on the start, which the batch entry holds.
    BatchPlan &pp = ctx->pure;
    if (pp.d_batch && pp.ids.size() == 1 && pp.ids[0] == walk && pp.fixed_n == n_lmt) {
        if (pp.fixed_start != start) {
            pp.fixed_start = start;      // the copy's source outlives the call
            HIP_TRY(ctx, hipMemcpyAsync(reinterpret_cast<char *>(pp.d_batch) + offsetof(BatchEntry, start),
                                        &pp.fixed_start, sizeof(uint32_t), hipMemcpyHostToDevice, ctx->stream));
        }
    } else {
        const psl_status st = make_plan(ctx, pp, &walk, 1, n_lmt, start);
        if (st) return st;
    }
    const Tables tabs = tables_of(ctx);
    HIP_TRY(ctx, launch_suffix(ctx->d_walks, ctx->pure.d_batch, 1, h.L, tabs, 0, &ctx->pure.seg, nullptr,
                               ctx->pure.shape.waves >= kEvalWavesMax,
                               ctx->stream));
    if (ctx->pure.split)
        HIP_TRY(ctx, launch_split_prep(ctx->d_walks, ctx->pure.d_batch, 1, tabs, ctx->pure.seg, ctx->stream));
    HIP_TRY(ctx, launch_eval(ctx->d_walks, ctx->pure.d_batch, ctx->pure.d_items, ctx->pure.n_items,
                             tabs, ctx->pure.shape, ctx->pure.d_queues, ctx->stream));
    if (ctx->pure.split)
        HIP_TRY(ctx, launch_lin(ctx->d_walks, ctx->pure.d_batch, ctx->pure.d_litems, ctx->pure.n_litems,
                                ctx->stream));
    HIP_TRY(ctx, launch_select(ctx->d_walks, ctx->pure.d_batch, 1, ctx->pure.comb_blocks, ctx->pure.comb_group, tabs, 1,
                               ctx->d_choice, nullptr, ctx->pure.d_done, ctx->amb_margin, ctx->stream));
    if (F_dev)
        HIP_TRY(ctx, hipMemcpyAsync(F_dev, ctx->pure.d_f, sizeof(double) * n_lmt,
                                    hipMemcpyDeviceToDevice, ctx->stream));
    if (psl_dev)
        HIP_TRY(ctx, hipMemcpyAsync(psl_dev, ctx->pure.d_p, sizeof(int32_t) * n_lmt,
                                    hipMemcpyDeviceToDevice, ctx->stream));
    std::vector<char> host(choice_dev_size());
    HIP_TRY(ctx, hipMemcpyAsync(host.data(), ctx->d_choice, host.size(), hipMemcpyDeviceToHost,
                                ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (out) {
        memset(out, 0, sizeof *out);
        choice_dev_unpack(host.data(), &out->i_best, &out->j_best, &out->F_best, &out->F_min,
                          &out->j_psl, &out->psl_min, &out->psl_k, &out->flags);
    }
    return PSL_OK;
}

psl_status psl_eval_neighbourhood_noalloc(psl_ctx *ctx, uint32_t walk, uint32_t start, uint32_t n_lmt,
                                          double *F_dev, int32_t *psl_dev, psl_choice *out)
{
    if (!ctx) return PSL_E_INVAL;
    if (serve_active(ctx)) return fail(ctx, PSL_E_STATE, "the context is serving");
    if (!walk_ok(ctx, walk)) return fail(ctx, PSL_E_STATE, "unknown walk %u", walk);
    const WalkHost &h = ctx->walks[walk];
    if (n_lmt < 1 || n_lmt > h.L || start >= h.L)
        return fail(ctx, PSL_E_INVAL, "start=%u n_lmt=%u for L=%u", start, n_lmt, h.L);
    if (!F_dev || !psl_dev) return fail(ctx, PSL_E_INVAL, "F_dev and psl_dev are required");
    if (!ctx->noalloc_scratch)
        return fail(ctx, PSL_E_STATE, "no fixed scratch on this device (%s)", ctx->noalloc_err.c_str());
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    // the plan's arrays and the choice record from the device's fixed scratch
    PlanMem mem;
    mem.base = (char *)ctx->noalloc_scratch;
    mem.cap = kNoAllocScratchBytes;
    mem.used = 256;                  // the choice record
    mem.F = F_dev;
    mem.P = psl_dev;
    void *d_choice = mem.base;
    BatchPlan pl;
    psl_status st = make_plan(ctx, pl, &walk, 1, n_lmt, start, nullptr, 0, &mem);
    if (st) {
        plan_free(ctx, pl);
        return st;
    }
    const Tables tabs = tables_of(ctx);
    HIP_TRY(ctx, launch_suffix(ctx->d_walks, pl.d_batch, 1, h.L, tabs, 0, &pl.seg, nullptr,
                               pl.shape.waves >= kEvalWavesMax, ctx->stream));
    HIP_TRY(ctx, launch_eval(ctx->d_walks, pl.d_batch, pl.d_items, pl.n_items, tabs, pl.shape, pl.d_queues,
                             ctx->stream));
    HIP_TRY(ctx, launch_select(ctx->d_walks, pl.d_batch, 1, pl.comb_blocks, pl.comb_group, tabs, 1, d_choice,
                               nullptr, pl.d_done, ctx->amb_margin, ctx->stream));
    alignas(16) unsigned char host[256];
    if (choice_dev_size() > sizeof host) return fail(ctx, PSL_E_STATE, "choice record too large");
    HIP_TRY(ctx, hipMemcpyAsync(host, d_choice, choice_dev_size(), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    plan_free(ctx, pl);
    if (out) {
        memset(out, 0, sizeof *out);
        choice_dev_unpack(host, &out->i_best, &out->j_best, &out->F_best, &out->F_min, &out->j_psl,
                          &out->psl_min, &out->psl_k, &out->flags);
    }
    return PSL_OK;
}

psl_status psl_apply_flip(psl_ctx *ctx, uint32_t walk, uint32_t j)
{
    if (!ctx) return PSL_E_INVAL;
    if (serve_active(ctx)) return fail(ctx, PSL_E_STATE, "the context is serving");
    if (!walk_ok(ctx, walk)) return fail(ctx, PSL_E_STATE, "unknown walk %u", walk);
    const WalkHost &h = ctx->walks[walk];
    if (j >= h.L) return fail(ctx, PSL_E_INVAL, "j=%u >= L=%u", j, h.L);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (const psl_status st = one_entry(ctx)) return st;
    BatchEntry e;
    memset(&e, 0, sizeof e);
    e.slot = walk;
    hipError_t r = hipMemcpy(ctx->d_one, &e, sizeof e, hipMemcpyHostToDevice);
    const Tables tabs = tables_of(ctx);
    if (r == hipSuccess) r = launch_apply(ctx->d_walks, ctx->d_one, seg_uniform(1, h.L), (int64_t)j, ctx->stream);
    if (r == hipSuccess) r = launch_flip_bit(ctx->d_walks, ctx->d_one, j, ctx->stream);
    if (r == hipSuccess) r = launch_fitness(ctx->d_walks, ctx->d_one, 1, tabs, 2, ctx->stream);
    if (r == hipSuccess) r = hipStreamSynchronize(ctx->stream);
    if (r != hipSuccess) return fail(ctx, PSL_E_HIP, "apply_flip: %s", hipGetErrorString(r));
    return PSL_OK;
}

psl_status psl_step_batch(psl_ctx *ctx, const uint32_t *walk_ids, uint32_t n, uint32_t steps,
                          uint32_t flags)
{
    if (!ctx) return PSL_E_INVAL;
    if (serve_active(ctx)) return fail(ctx, PSL_E_STATE, "the context is serving");
    if (n == 0 || steps == 0) return PSL_OK;
    if (!walk_ids) return fail(ctx, PSL_E_INVAL, "walk_ids is NULL");
    std::vector<uint32_t> sorted(walk_ids, walk_ids + n);
    std::sort(sorted.begin(), sorted.end());
    for (uint32_t b = 0; b < n; ++b) {
        if (!walk_ok(ctx, sorted[b])) return fail(ctx, PSL_E_STATE, "unknown walk %u", sorted[b]);
        if (b && sorted[b] == sorted[b - 1]) return fail(ctx, PSL_E_INVAL, "walk %u repeated", sorted[b]);
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    psl_status st = PSL_OK;
    size_t hit = ctx->plans.size();
    for (size_t x = 0; x < ctx->plans.size(); ++x) {
        const BatchPlan &c = ctx->plans[x];
        if (c.ids.size() == n && std::equal(walk_ids, walk_ids + n, c.ids.begin())) hit = x;
    }
    if (hit == ctx->plans.size()) {
        if (ctx->plans.size() >= kPlanCache) {
            HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
            plan_free(ctx, ctx->plans.front());
            ctx->plans.erase(ctx->plans.begin());
        }
        ctx->plans.emplace_back();
        if ((st = make_plan(ctx, ctx->plans.back(), walk_ids, n, UINT32_MAX, 0))) {
            plan_free(ctx, ctx->plans.back());
            ctx->plans.pop_back();
            return st;
        }
    } else if (hit + 1 != ctx->plans.size()) {
        std::rotate(ctx->plans.begin() + hit, ctx->plans.begin() + hit + 1, ctx->plans.end());
    }
    BatchPlan &pl = ctx->plans.back();
    const Tables tabs = tables_of(ctx);
    if ((flags & PSL_STEP_GRAPH) && !ctx->timing) {
        if (!pl.gexec && (st = capture_step(ctx, pl, tabs, n))) return st;
        for (uint32_t s = 0; s < steps; ++s) HIP_TRY(ctx, hipGraphLaunch(pl.gexec, ctx->stream));
    } else {
        for (uint32_t s = 0; s < steps; ++s)
            if ((st = launch_step(ctx, pl, tabs, n, ctx->timing))) return st;
    }
    if (flags & PSL_STEP_BLOCKING) HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return PSL_OK;
}

psl_status psl_read_walk(psl_ctx *ctx, uint32_t walk, psl_walk_state *out, uint64_t *pivot_bits,
                         uint64_t *local_best_bits, uint64_t *best_bits, int32_t *C)
{
    if (!ctx) return PSL_E_INVAL;
    if (serve_active(ctx)) return fail(ctx, PSL_E_STATE, "the context is serving");
    if (!walk_ok(ctx, walk)) return fail(ctx, PSL_E_STATE, "unknown walk %u", walk);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    WalkDev w;
    HIP_TRY(ctx, hipMemcpy(&w, ctx->d_walks + walk, sizeof w, hipMemcpyDeviceToHost));
    if (pivot_bits) HIP_TRY(ctx, hipMemcpy(pivot_bits, w.pivot, 8 * w.nw, hipMemcpyDeviceToHost));
    if (local_best_bits)
        HIP_TRY(ctx, hipMemcpy(local_best_bits, w.local_best, 8 * w.nw, hipMemcpyDeviceToHost));
    if (best_bits) HIP_TRY(ctx, hipMemcpy(best_bits, w.best, 8 * w.nw, hipMemcpyDeviceToHost));
    if (C) HIP_TRY(ctx, hipMemcpy(C, w.C, sizeof(int32_t) * w.L, hipMemcpyDeviceToHost));
    if (out) {
        memset(out, 0, sizeof *out);
        out->L = w.L;
        out->alpha1 = w.alpha1;
        out->alpha2 = w.alpha2;
        out->alpha = w.alpha;
        out->n_lmt = w.n_lmt;
        out->ls_lmt = w.ls_lmt;
        out->flip_lmt = w.flip_lmt;
        out->switch_period = w.switch_period;
        out->seed = w.seed;
        out->t = w.t;
        out->q = w.q;
        out->value_local = w.value_local;
        out->F_pivot = w.F_pivot;
        out->psl_pivot = w.psl_pivot;
        out->psl_best = w.psl_best;
        out->unimproved = w.unimproved;
        out->last_k = w.k;
        out->last_value_step = w.value_step;
        out->last_start = w.start;
        out->last_flags = w.flags;
    }
    return PSL_OK;
}

psl_status psl_timing_enable(psl_ctx *ctx, int on)
{
    if (!ctx) return PSL_E_INVAL;
    if (serve_active(ctx)) return fail(ctx, PSL_E_STATE, "the context is serving");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    timing_drop(ctx);
    ctx->timing = on != 0;
    ctx->eval_ms = ctx->rest_ms = ctx->prep_ms = ctx->lin_ms = 0.0;
    ctx->eval_launches = ctx->steps_timed = 0;
    return PSL_OK;
}

psl_status psl_timing_read(psl_ctx *ctx, psl_timing *out)
{
    if (!ctx || !out) return PSL_E_INVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    psl_status st = timing_collect(ctx);
    if (st) return st;
    out->eval_ms = ctx->eval_ms;
    out->eval_launches = ctx->eval_launches;
    out->rest_ms = ctx->rest_ms;
    out->steps = ctx->steps_timed;
    out->prep_ms = ctx->prep_ms;
    out->lin_ms = ctx->lin_ms;
    return PSL_OK;
}

psl_status psl_autotune(psl_ctx *ctx, const uint32_t *walk_ids, uint32_t n, psl_tune_choice *out)
{
    if (!ctx) return PSL_E_INVAL;
    if (serve_active(ctx)) return fail(ctx, PSL_E_STATE, "the context is serving");
    if (n == 0 || !walk_ids) return fail(ctx, PSL_E_INVAL, "empty batch");
    for (uint32_t b = 0; b < n; ++b)
        if (!walk_ok(ctx, walk_ids[b])) return fail(ctx, PSL_E_STATE, "unknown walk %u", walk_ids[b]);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    std::vector<uint32_t> Ls(n), nl(n);
    for (uint32_t b = 0; b < n; ++b) {
        Ls[b] = ctx->walks[walk_ids[b]].L;
        nl[b] = ctx->walks[walk_ids[b]].n_lmt;
    }
    const uint32_t key = tune_key(Ls.data(), nl.data(), n);
    ctx->tuned.erase(key);
    ctx->tuned_items.erase(key);
    const EvalShape def = pick_shape(ctx, Ls.data(), nl.data(), n);
    std::vector<EvalShape> cands;
    for (int waves : {kEvalWavesMax, kEvalWaves, kEvalWavesSmall}) {
        EvalShape f;
        f.waves = waves;
        cands.push_back(f);
        for (uint32_t bpc = 1; bpc <= max_blocks_per_cu(waves); ++bpc) {
            EvalShape q;
            q.waves = waves;
            q.persistent = 1;
            q.grid = bpc * ctx->n_cu;
            cands.push_back(q);
        }
    }
    const Tables tabs = tables_of(ctx);
    hipEvent_t e0, e1;
    HIP_TRY(ctx, hipEventCreate(&e0));
    HIP_TRY(ctx, hipEventCreate(&e1));
    // mean time of one evaluation launch in a given shape and work-item target
    auto time_eval = [&](const EvalShape &c, uint32_t items, double &avg) -> psl_status {
        BatchPlan tmp;
        psl_status s2 = make_plan(ctx, tmp, walk_ids, n, UINT32_MAX, 0, &c, items);
        if (s2) return s2;
        hipError_t e = launch_suffix(ctx->d_walks, tmp.d_batch, n, tmp.max_L, tabs, 0, &tmp.seg, nullptr,
                                     tmp.shape.waves >= kEvalWavesMax, ctx->stream);
        if (e == hipSuccess)   // warm-up
            e = launch_eval(ctx->d_walks, tmp.d_batch, tmp.d_items, tmp.n_items, tabs, tmp.shape,
                            tmp.d_queues, ctx->stream);
        const int reps = 2;
        if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r)
            e = launch_eval(ctx->d_walks, tmp.d_batch, tmp.d_items, tmp.n_items, tabs, tmp.shape,
                            tmp.d_queues, ctx->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        plan_free(ctx, tmp);
        if (e != hipSuccess) return fail(ctx, PSL_E_HIP, "autotune: %s", hipGetErrorString(e));
        avg = ms / reps;
        return PSL_OK;
    };
    double best_ms = 1e300, def_ms = 0.0;
    EvalShape best = def;
    uint32_t best_items = ctx->eval_items;
    psl_status st = PSL_OK;
    for (const EvalShape &c : cands) {
        double avg = 0.0;
        if ((st = time_eval(c, ctx->eval_items, avg))) break;
        if (c.waves == def.waves && c.persistent == def.persistent && c.grid == def.grid) def_ms = avg;
        if (avg < best_ms) {
            best_ms = avg;
            best = c;
        }
    }
    // then the work-item target for that shape: half, twice and four times
    // the context's value
    if (!st) {
        for (const uint64_t f : {1ull, 4ull, 8ull}) {       // x/2, 2x, 4x of the value
            const uint32_t items = (uint32_t)std::min<uint64_t>(
                kEvalItemsMax, std::max<uint64_t>(1, (uint64_t)ctx->eval_items * f / 2));
            if (items == ctx->eval_items) continue;
            double avg = 0.0;
            if ((st = time_eval(best, items, avg))) break;
            if (avg < best_ms) {
                best_ms = avg;
                best_items = items;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    ctx->tuned[key] = best;
    ctx->tuned_items[key] = best_items;
    plans_clear(ctx);            // later plans pick up the choice
    if (out) {
        memset(out, 0, sizeof *out);
        out->waves = best.waves;
        out->persistent = best.persistent;
        out->blocks_per_cu = best.persistent ? (int32_t)(best.grid / ctx->n_cu) : 0;
        out->eval_items = (int32_t)best_items;
        out->eval_ms = best_ms;
        out->default_ms = def_ms;
    }
    return PSL_OK;
}

psl_status psl_tune_save(psl_ctx *ctx, const char *path)
{
    if (!ctx || !path) return PSL_E_INVAL;
    FILE *f = fopen(path, "w");
    if (!f) return fail(ctx, PSL_E_INVAL, "cannot write %s", path);
    for (const auto &kv : ctx->tuned) {
        auto it = ctx->tuned_items.find(kv.first);
        fprintf(f, "%u %d %d %u %u\n", kv.first, kv.second.waves, kv.second.persistent,
                kv.second.persistent ? kv.second.grid / ctx->n_cu : 0u,
                it != ctx->tuned_items.end() ? it->second : ctx->eval_items);
    }
    fclose(f);
    return PSL_OK;
}

psl_status psl_tune_load(psl_ctx *ctx, const char *path)
{
    if (!ctx || !path) return PSL_E_INVAL;
    if (serve_active(ctx)) return fail(ctx, PSL_E_STATE, "the context is serving");
    FILE *f = fopen(path, "r");
    if (!f) return fail(ctx, PSL_E_INVAL, "cannot read %s", path);
    std::map<uint32_t, EvalShape> got;
    std::map<uint32_t, uint32_t> got_items;
    char line[256];
    while (fgets(line, sizeof line, f)) {
        unsigned key, bpc, items = 0;
        int waves, pers;
        char extra;
        const int r = sscanf(line, "%u %d %d %u %u %c", &key, &waves, &pers, &bpc, &items, &extra);
        if (r <= 0) continue;                   // blank line
        if ((r != 4 && r != 5) || (waves != kEvalWavesMax && waves != kEvalWaves && waves != kEvalWavesSmall) ||
            (pers != 0 && pers != 1) || (pers && (bpc < 1 || bpc > max_blocks_per_cu(waves))) ||
            (r == 5 && (items < 1 || items > kEvalItemsMax))) {
            fclose(f);
            return fail(ctx, PSL_E_INVAL, "bad tuning line in %s", path);
        }
        EvalShape sh;
        sh.waves = waves;
        sh.persistent = pers;
        sh.grid = pers ? bpc * ctx->n_cu : 0;
        got[key] = sh;
        if (r == 5) got_items[key] = items;
    }
    fclose(f);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (auto &kv : got) ctx->tuned[kv.first] = kv.second;
    for (auto &kv : got_items) ctx->tuned_items[kv.first] = kv.second;
    plans_clear(ctx);
    return PSL_OK;
}

psl_status psl_set_option(psl_ctx *ctx, int option, int64_t value)
{
    if (!ctx) return PSL_E_INVAL;
    if (serve_active(ctx)) return fail(ctx, PSL_E_STATE, "the context is serving");
    const bool ok = (option == PSL_OPT_NEAR_LIMIT && value >= -1) ||
                    (option == PSL_OPT_EVAL_ITEMS && (value == -1 || (value >= 1 && value <= kEvalItemsMax))) ||
                    (option == PSL_OPT_AMBIG_MARGIN && value >= -1 && value <= kAmbigMarginMax) ||
                    (option == PSL_OPT_SPLIT && value >= -1 && value <= 2) ||
                    (option == PSL_OPT_TEST_FAIL_ADMIT && value >= 0 && value <= UINT32_MAX);
    if (!ok) return fail(ctx, PSL_E_INVAL, "option %d value %lld", option, (long long)value);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (option == PSL_OPT_NEAR_LIMIT)
        ctx->near_limit = value;
    else if (option == PSL_OPT_EVAL_ITEMS)
        ctx->eval_items = value < 0 ? kEvalItemsDefault : (uint32_t)value;
    else if (option == PSL_OPT_AMBIG_MARGIN)
        ctx->amb_margin = value < 0 ? kAmbigMarginDefault : (double)value * 1e-15;
    else if (option == PSL_OPT_SPLIT)
        ctx->split_mode = value < 0 ? 2 : (int)value;
    else
        ctx->test_fail_admit = (uint32_t)value;
    plans_clear(ctx);            // cached layouts carry the old value
    return PSL_OK;
}

psl_status psl_trace_enable(psl_ctx *ctx, uint32_t walk, uint32_t capacity)
{
    if (!ctx) return PSL_E_INVAL;
    if (serve_active(ctx)) return fail(ctx, PSL_E_STATE, "the context is serving");
    if (!walk_ok(ctx, walk)) return fail(ctx, PSL_E_STATE, "unknown walk %u", walk);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    WalkHost &h = ctx->walks[walk];
    void *ring = nullptr;
    if (capacity) {
        psl_status st = dev_alloc(ctx, &ring, sizeof(TraceEntry) * capacity, false);
        if (st) return st;
    }
    WalkDev w;
    HIP_TRY(ctx, hipMemcpy(&w, ctx->d_walks + walk, sizeof w, hipMemcpyDeviceToHost));
    w.trace = (TraceEntry *)ring;
    w.trace_cap = capacity;
    HIP_TRY(ctx, hipMemcpy(ctx->d_walks + walk, &w, sizeof w, hipMemcpyHostToDevice));
    dev_free(ctx, h.trace, false);
    h.trace = ring;
    return PSL_OK;
}

psl_status psl_trace_read(psl_ctx *ctx, uint32_t walk, psl_trace_entry *out, uint32_t max_entries,
                          uint32_t *n_out)
{
    if (!ctx || !n_out || (max_entries && !out)) return PSL_E_INVAL;
    if (serve_active(ctx)) return fail(ctx, PSL_E_STATE, "the context is serving");
    if (!walk_ok(ctx, walk)) return fail(ctx, PSL_E_STATE, "unknown walk %u", walk);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    WalkDev w;
    HIP_TRY(ctx, hipMemcpy(&w, ctx->d_walks + walk, sizeof w, hipMemcpyDeviceToHost));
    if (!w.trace_cap) return fail(ctx, PSL_E_STATE, "walk %u has no trace", walk);
    std::vector<TraceEntry> ring(w.trace_cap);
    HIP_TRY(ctx, hipMemcpy(ring.data(), w.trace, sizeof(TraceEntry) * w.trace_cap, hipMemcpyDeviceToHost));
    const uint64_t have = std::min<uint64_t>(w.t, w.trace_cap);
    const uint64_t n = std::min<uint64_t>(have, max_entries);
    for (uint64_t x = 0; x < n; ++x) {
        const uint64_t t = w.t - n + x;
        const TraceEntry &e = ring[t % w.trace_cap];
        psl_trace_entry &o = out[x];
        o.t = e.t;
        o.start = e.start;
        o.k = e.k;
        o.value_step = e.value_step;
        o.psl_k = e.psl_k;
        o.psl_best = e.psl_best;
        o.alpha = e.alpha;
        o.flags = e.flags;
    }
    *n_out = (uint32_t)n;
    return PSL_OK;
}

psl_status psl_restore_walk(psl_ctx *ctx, uint32_t walk, const psl_walk_state *st, const uint64_t *pivot,
                            const uint64_t *local_best, const uint64_t *best)
{
    if (!ctx) return PSL_E_INVAL;
    if (serve_active(ctx)) return fail(ctx, PSL_E_STATE, "the context is serving");
    if (!walk_ok(ctx, walk)) return fail(ctx, PSL_E_STATE, "unknown walk %u", walk);
    if (!st || !pivot || !local_best || !best) return fail(ctx, PSL_E_INVAL, "null argument");
    WalkHost &h = ctx->walks[walk];
    psl_walk_cfg c;
    memset(&c, 0, sizeof c);
    c.L = st->L;
    c.alpha1 = st->alpha1;
    c.alpha2 = st->alpha2;
    c.n_lmt = st->n_lmt;
    c.ls_lmt = st->ls_lmt;
    c.flip_lmt = st->flip_lmt;
    c.switch_period = st->switch_period;
    c.seed = st->seed;
    psl_status s2 = check_cfg(ctx, &c);
    if (s2) return s2;
    if (st->L != h.L) return fail(ctx, PSL_E_INVAL, "state of L=%u for a walk of L=%u", st->L, h.L);
    if (st->alpha != st->alpha1 && st->alpha != st->alpha2) return fail(ctx, PSL_E_INVAL, "alpha");
    const uint32_t nw = h.nw, L = h.L;
    if ((L & 63u) && ((pivot[nw - 1] | local_best[nw - 1] | best[nw - 1]) >> (L & 63u)))
        return fail(ctx, PSL_E_INVAL, "bits set at or beyond L");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    WalkDev w;
    HIP_TRY(ctx, hipMemcpy(&w, ctx->d_walks + walk, sizeof w, hipMemcpyDeviceToHost));
    w.seed = st->seed;
    w.alpha1 = st->alpha1;
    w.alpha2 = st->alpha2;
    w.alpha = st->alpha;
    w.n_lmt = st->n_lmt ? st->n_lmt : L;
    w.ls_lmt = st->ls_lmt;
    w.flip_lmt = st->flip_lmt;
    w.switch_period = st->switch_period;
    w.t = st->t;
    w.q = st->q;
    w.value_local = st->value_local;
    w.psl_best = st->psl_best;
    w.unimproved = st->unimproved;
    w.pending = 0;
    w.n_flips = 0;
    w.flags = 0;
    HIP_TRY(ctx, hipMemcpy(ctx->d_walks + walk, &w, sizeof w, hipMemcpyHostToDevice));
    h.n_lmt = w.n_lmt;
    h.flip_lmt = w.flip_lmt;
    plans_clear(ctx);            // N_lmt may differ
    // C of local_best (and C) from local_best's bits, then C from the pivot's
    if (const psl_status rs = one_entry(ctx)) return rs;
    BatchEntry e;
    memset(&e, 0, sizeof e);
    e.slot = walk;
    hipError_t r = hipMemcpy(ctx->d_one, &e, sizeof e, hipMemcpyHostToDevice);
    const Tables tabs = tables_of(ctx);
    if (r == hipSuccess) r = hipMemcpy(w.pivot, local_best, 8ull * nw, hipMemcpyHostToDevice);
    if (r == hipSuccess) r = launch_corr(ctx->d_walks, ctx->d_one, 1, L, 0, ctx->stream);
    if (r == hipSuccess) r = hipStreamSynchronize(ctx->stream);
    if (r == hipSuccess) r = hipMemcpy(w.pivot, pivot, 8ull * nw, hipMemcpyHostToDevice);
    if (r == hipSuccess) r = hipMemcpy(w.local_best, local_best, 8ull * nw, hipMemcpyHostToDevice);
    if (r == hipSuccess) r = hipMemcpy(w.best, best, 8ull * nw, hipMemcpyHostToDevice);
    if (r == hipSuccess) r = launch_corr(ctx->d_walks, ctx->d_one, 1, L, 2, ctx->stream);
    if (r == hipSuccess) r = launch_fitness(ctx->d_walks, ctx->d_one, 1, tabs, 2, ctx->stream);
    if (r == hipSuccess) r = hipStreamSynchronize(ctx->stream);
    if (r != hipSuccess) return fail(ctx, PSL_E_HIP, "restore: %s", hipGetErrorString(r));
    return PSL_OK;
}

psl_status psl_eval_shape(psl_ctx *ctx, uint32_t L, uint32_t n_lmt, uint32_t n_walks,
                          uint32_t *cand_tiles, uint32_t *k_splits)
{
    (void)ctx;
    if (L < 2 || L > PSL_L_MAX || n_lmt < 1 || n_lmt > L || n_walks < 1 || n_walks > (1u << 20) || !cand_tiles ||
        !k_splits)
        return PSL_E_INVAL;
    // the shape a batch of n_walks such walks is launched with
    const std::vector<uint32_t> Ls(n_walks, L), nl(n_walks, n_lmt);
    const uint32_t tile = 64u * (ctx ? pick_shape(ctx, Ls.data(), nl.data(), n_walks).waves
                                     : eval_waves(nl.data(), n_walks));
    const uint32_t tiles = (n_lmt + tile - 1) / tile;
    const uint64_t W = (uint64_t)tiles * (L - 1) * n_walks;
    const uint32_t K = item_shifts_for(W, tile, ctx ? ctx->eval_items : kEvalItemsDefault);
    eval_shape_k(L, n_lmt, K, tile, cand_tiles, k_splits);
    return PSL_OK;
}

}  // extern "C"
