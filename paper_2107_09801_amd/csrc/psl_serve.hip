// psl_serve.hip -- the request loop of libpsl (psl_serve_* in include/psl.h).
//
// One host thread owns the context's stream while serving. Each iteration it
//   1. takes submitted jobs into a FIFO,
//   2. finishes retiring jobs whose read-back has landed,
//   3. admits jobs from the FIFO head while the HBM budget and slots allow
//      (zeroed slab, walk record, then one batched init launch),
//   4. advances every admitted walk by one step of Algorithm 1 with the same
//      launch sequence psl_step_batch uses (the batch is whatever is admitted:
//      continuous batching), and
//   5. retires the walks that reached their budget: their record and best
//      sequence are copied to pinned host memory behind an event, and their
//      slot is released (later reuse is ordered after the copy on the same
//      stream); the slab is freed later, with others, after a stream sync.
// Device memory: each walk slab is an allocation of its own, of its size
// class; retired slabs wait in a pool, where a later job of the same class
// takes one over (the stream orders its use after the retired walk's
// read-back), until the pool is freed. The scratch buffers of the batch and
// of admissions grow and shrink within the sum of the admitted jobs' scratch
// bounds (plus kServeFixed). A job is admitted while the admitted jobs'
// footprints (slab class + scratch bound), the pooled slabs and any scratch
// beyond that sum fit in hbm_budget, so the loop's device memory stays within
// hbm_budget + kServeFixed.
// No step waits on the host: at most two iterations are in flight, and the
// host only waits for the iteration two back before reusing its staging.
#include "psl_internal.h"

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>

using namespace psl;

namespace psl_rt {

namespace {

uint64_t now_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Largest k-splits x candidates, and k-splits x candidate tiles, a walk of
// length L with n_lmt candidates gets in any batch: a batch's work only
// lengthens the work items, so the walk alone with the largest work-item
// target items_cap bounds both, over the three tile widths.
void split_bound(uint32_t L, uint32_t n_lmt, uint32_t items_cap, uint64_t *ks_n, uint64_t *ks_tiles)
{
    *ks_n = 0;
    *ks_tiles = 0;
    for (int waves : {kEvalWavesSmall, kEvalWaves, kEvalWavesMax}) {
        const uint32_t tile = 64u * (uint32_t)waves;
        const uint64_t tiles = (n_lmt + tile - 1) / tile;
        const uint32_t K = item_shifts_for(tiles * (L - 1), tile, items_cap);
        uint32_t t = 0, ks = 0;
        eval_shape_k(L, n_lmt, K, tile, &t, &ks);
        *ks_n = std::max<uint64_t>(*ks_n, (uint64_t)ks * n_lmt);
        *ks_tiles = std::max<uint64_t>(*ks_tiles, (uint64_t)ks * t);
    }
}

// Upper bound of one walk's share of the scratch buffers of any batch and
// admission it is in.
size_t scratch_bound(uint32_t L, uint32_t n_lmt, uint32_t items_cap)
{
    uint64_t ks_n = 0, ks_tiles = 0;
    split_bound(L, n_lmt, items_cap, &ks_n, &ks_tiles);
    const uint64_t segs = seg_count(L, kSegShiftMin);
    return (size_t)(12ull * ks_n                           // partial sums and maxima
                    + 12ull * n_lmt                        // F and PSL per candidate
                    + 24ull * suffix_len(L)                // chunk suffix arrays: step, admission
                    + 4ull * (kNearCap + 1)                // near-peak list
                    + sizeof(SelPart) * kCombMaxBlocks     // combine-block minima
                    + 2 * sizeof(BatchEntry) + 32          // batch and admission entries, list slots
                    + sizeof(EvalItem) * 8 * ks_tiles      // work items, with the flat form's padding
                    + 12ull * segs);                       // per-segment totals of the O(L) passes
}

// Scratch capacity beyond the jobs' bounds: the buffers' smallest size
// (kMinCap elements each) and the queue record.
constexpr size_t kMinCap = 1024;
constexpr size_t kServeFixed = (size_t)1 << 20;
// The slab pool is freed once it holds this many slabs (or bytes).
constexpr size_t kFlushSlabs = 1024;
constexpr size_t kFlushBytes = (size_t)256 << 20;

// Slab allocation size: 4 KiB steps up to 64 KiB, then eight classes per
// power of two (at most 1/8 more than the slab).
size_t slab_class(size_t bytes)
{
    if (bytes <= ((size_t)64 << 10)) return align_up(std::max<size_t>(bytes, 1), (size_t)4 << 10);
    size_t p = (size_t)64 << 10;
    while (2 * p <= bytes) p *= 2;
    return align_up(bytes, p / 8);
}

size_t job_footprint(const psl_walk_cfg &c, uint32_t items_cap)
{
    return slab_class(slab_layout(c.L).slab_bytes) + scratch_bound(c.L, c.n_lmt ? c.n_lmt : c.L, items_cap);
}

struct Job {
    uint64_t ticket = 0;
    psl_walk_cfg cfg{};
    uint64_t budget = 0;
    uint64_t *best_out = nullptr;
    uint64_t t_arrive = 0, t_admit = 0;
    size_t foot = 0;          // slab + scratch bound, counted against the budget
    size_t bound = 0;         // scratch bound
    uint32_t slot = UINT32_MAX;
    void *slab = nullptr;
    WalkDev dev{};            // device pointers of the walk
    uint64_t steps = 0;
    char *host = nullptr;     // pinned read-back: WalkDev, then best bits
    size_t host_bytes = 0;
    hipEvent_t ev = nullptr;
};

// Grow-only device buffer.
template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t cap = 0;
};

}  // namespace

struct Server {
    psl_serve_cfg cfg{};
    psl_ctx *ctx = nullptr;
    std::thread th;
    // shared with submitters (mu)
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false, drain = false, running = false;
    std::deque<Job> incoming;
    std::map<uint64_t, psl_job_result> done;
    std::map<uint64_t, int> live;               // tickets queued, running or retiring
    uint64_t next_ticket = 1;
    psl_serve_stats stats{};
    // scheduler-owned
    std::deque<Job> pending;
    std::vector<Job> active, retiring;
    size_t used = 0;              // footprints of the admitted jobs
    size_t bounds = 0;            // their scratch bounds
    uint32_t items_cap = 0;       // largest work-item target of the context
    size_t dev_scratch = 0;       // capacity of the scratch buffers, bytes
    std::multimap<size_t, void *> to_free;     // retired slabs by size class
    size_t to_free_bytes = 0;
    DevBuf<BatchEntry> d_batch, d_admit;
    DevBuf<EvalItem> d_items;
    DevBuf<double> d_fpart, d_f, d_s0;
    DevBuf<uint32_t> d_mpart, d_m0, d_near, d_want;
    DevBuf<SelPart> d_red;
    DevBuf<uint32_t> d_pend;      // pending list of the iteration's batch
    DevBuf<uint32_t> d_done;      // per batch position: combine blocks finished (0 between launches)
    DevBuf<uint32_t> d_seg, d_adm_seg;   // segment maps (batch, admitted walks)
    DevBuf<double> d_segtot;             // per segment of the batch map: chunk-sum total
    DevBuf<uint32_t> d_segmax;
    SegMap seg{};
    DevBuf<double> d_adm_s0;      // chunk arrays of the admitted walks' fitness pass
    DevBuf<uint32_t> d_adm_m0;
    uint32_t comb_blocks = 1, comb_group = 1;
    DevBuf<int32_t> d_p;
    uint32_t n_items = 0, max_L = 0;
    EvalShape shape;
    DevBuf<EvalQueues> d_queues;
    bool dirty = true;
    // pinned staging, two halves used by alternate iterations
    char *stage[2] = {nullptr, nullptr};
    size_t stage_cap[2] = {0, 0};
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    bool stage_used[2] = {false, false};
    int cur = 0;
    std::multimap<size_t, char *> pinned_free;  // read-back buffers by size
    uint64_t busy_from = 0;

    void run();
    psl_status ensure_stage(size_t need);
    psl_status iterate();
    psl_status upload_layout(char *&sp, char *stage_end);
    psl_status admit(char *&sp, char *stage_end);
    psl_status admit_start(std::vector<Job> &adm, char *&sp, char *stage_end);
    uint32_t n_admissions = 0;    // admissions that took jobs (test hook count)
    void retire_finished();
    void fail_all(int32_t status);
    void finish(Job &j, int32_t status);
    // scratch beyond what the admitted jobs' bounds allow
    size_t scratch_over() const
    {
        const size_t allow = bounds + kServeFixed;
        return dev_scratch > allow ? dev_scratch - allow : 0;
    }
    psl_status flush_free();
    psl_status release_scratch();
    struct BufNeed {
        void **p;
        size_t *cap;
        size_t elem;
        size_t need;
    };
    template <class T>
    static BufNeed buf(DevBuf<T> &b, size_t n)
    {
        return BufNeed{(void **)&b.p, &b.cap, sizeof(T), n};
    }
    psl_status size_bufs(std::initializer_list<BufNeed> bufs);
    std::vector<BufNeed> all_bufs();
};

namespace {

template <class T>
void release(psl_ctx *ctx, DevBuf<T> &b)
{
    dev_free(ctx, b.p, false);
    b = DevBuf<T>();
}

psl_status pinned(psl_ctx *ctx, Server &s, size_t bytes, char **out)
{
    auto it = s.pinned_free.lower_bound(bytes);
    if (it != s.pinned_free.end() && it->first <= 2 * bytes) {
        *out = it->second;
        s.pinned_free.erase(it);
        return PSL_OK;
    }
    void *p = nullptr;
    HIP_TRY(ctx, hipHostMalloc(&p, bytes, hipHostMallocDefault));
    *out = (char *)p;
    return PSL_OK;
}

}  // namespace

void Server::finish(Job &j, int32_t status)
{
    psl_job_result r;
    memset(&r, 0, sizeof r);
    r.status = status;
    r.t_arrive_ns = j.t_arrive;
    r.t_admit_ns = j.t_admit;
    r.t_done_ns = now_ns();
    r.steps = j.steps;
    if (status == PSL_OK && j.host) {
        WalkDev w;
        memcpy(&w, j.host, sizeof w);
        r.psl_best = w.psl_best;
        r.psl_final = w.psl_pivot;
        r.alpha_final = w.alpha;
        r.F_final = w.F_pivot;
        r.steps = w.t;
        if (j.best_out) memcpy(j.best_out, j.host + sizeof(WalkDev), 8ull * w.nw);
    }
    if (j.host) pinned_free.emplace(j.host_bytes, j.host);
    if (j.ev) (void)hipEventDestroy(j.ev);
    j.host = nullptr;
    j.ev = nullptr;
    std::lock_guard<std::mutex> g(mu);
    done[j.ticket] = r;
    live.erase(j.ticket);
    if (status == PSL_OK) stats.completed++;
    else stats.failed++;
}

void Server::fail_all(int32_t status)
{
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipGetLastError();
    for (auto &j : retiring) finish(j, status);
    retiring.clear();
    for (auto &j : active) {
        dev_free(ctx, j.slab, false);
        j.slab = nullptr;
        if (j.slot != UINT32_MAX) {
            ctx->walks[j.slot] = WalkHost();
            ctx->free_slots.push_back(j.slot);
        }
        finish(j, status);
    }
    active.clear();
    used = 0;
    bounds = 0;
    (void)flush_free();
    dirty = true;
}

// Frees the pooled slabs (their read-backs are queued before the sync).
psl_status Server::flush_free()
{
    if (to_free.empty()) return PSL_OK;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (auto &f : to_free) dev_free(ctx, f.second, false);
    to_free.clear();
    to_free_bytes = 0;
    return PSL_OK;
}

std::vector<Server::BufNeed> Server::all_bufs()
{
    return {buf(d_batch, 0),  buf(d_admit, 0),  buf(d_items, 0),   buf(d_fpart, 0),  buf(d_f, 0),
            buf(d_s0, 0),     buf(d_mpart, 0),  buf(d_m0, 0),      buf(d_near, 0),   buf(d_want, 0),
            buf(d_red, 0),    buf(d_pend, 0),   buf(d_done, 0),    buf(d_seg, 0),    buf(d_adm_seg, 0),
            buf(d_segtot, 0), buf(d_segmax, 0), buf(d_adm_s0, 0),  buf(d_adm_m0, 0), buf(d_p, 0),
            buf(d_queues, 0)};
}

// Frees every scratch buffer (they grow again with the next layout).
psl_status Server::release_scratch()
{
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (auto &b : all_bufs()) {
        dev_free(ctx, *b.p, false);
        *b.p = nullptr;
        *b.cap = 0;
    }
    dev_scratch = 0;
    dirty = true;
    return PSL_OK;
}

// Gives each listed buffer at least its need: 1.5 x the need when a buffer
// grows, or, when that would take the scratch past the admitted jobs' bounds,
// exactly the need (at least kMinCap), shrinking the listed buffers that hold
// more. A resize waits for the stream first (work queued earlier may still
// read the old buffer); contents are not kept.
psl_status Server::size_bufs(std::initializer_list<BufNeed> bufs)
{
    size_t grown = dev_scratch;
    bool any = false;
    for (const BufNeed &b : bufs) {
        if (b.need <= *b.cap) continue;
        any = true;
        grown += (std::max(b.need + b.need / 2, kMinCap) - *b.cap) * b.elem;
    }
    const bool tight = grown > bounds + kServeFixed;
    if (!any && !tight) return PSL_OK;
    bool synced = false;
    for (const BufNeed &b : bufs) {
        const size_t want = tight ? std::max(b.need, kMinCap)
                                  : (b.need <= *b.cap ? *b.cap : std::max(b.need + b.need / 2, kMinCap));
        if (want == *b.cap) continue;
        if (!synced) {
            HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
            synced = true;
        }
        dev_free(ctx, *b.p, false);
        dev_scratch -= *b.cap * b.elem;
        *b.p = nullptr;
        *b.cap = 0;
        void *q;
        const psl_status st = dev_alloc(ctx, &q, want * b.elem, false);
        if (st) return st;
        *b.p = q;
        *b.cap = want;
        dev_scratch += want * b.elem;
    }
    return PSL_OK;
}

void Server::retire_finished()
{
    for (size_t x = 0; x < retiring.size();) {
        if (hipEventQuery(retiring[x].ev) == hipSuccess) {
            finish(retiring[x], PSL_OK);
            retiring.erase(retiring.begin() + x);
        } else {
            ++x;
        }
    }
}

// Admits jobs from the FIFO head; their walk records and the batched init
// arrays go through the staging buffer.
psl_status Server::admit(char *&sp, char *stage_end)
{
    std::vector<Job> adm;
    psl_status st;
    while (!pending.empty()) {
        Job &j = pending.front();
        if (active.size() + adm.size() >= cfg.max_slots) break;
        // strict FIFO: no overtaking. Slabs awaiting their free and scratch
        // beyond the admitted jobs' bounds count too; both are given back
        // when that lets the job in.
        const size_t base = used + j.foot;
        if (base > cfg.hbm_budget) break;
        if (base + to_free_bytes + scratch_over() > cfg.hbm_budget) {
            if ((st = flush_free())) return st;
            if (base + scratch_over() > cfg.hbm_budget && adm.empty() && (st = release_scratch())) return st;
            if (base + scratch_over() > cfg.hbm_budget) break;
        }
        const size_t cls = slab_class(slab_layout(j.cfg.L).slab_bytes);
        void *slab = nullptr;
        auto pooled = to_free.find(cls);
        if (pooled != to_free.end()) {
            slab = pooled->second;
            to_free.erase(pooled);
            to_free_bytes -= cls;
        } else if (dev_alloc(ctx, &slab, cls, false) != PSL_OK) {
            if (!active.empty() || !adm.empty()) break;    // room comes back as jobs retire
            Job f = std::move(j);
            pending.pop_front();
            finish(f, PSL_E_NOMEM);
            continue;
        }
        j.slab = slab;
        used += j.foot;
        bounds += j.bound;
        adm.push_back(std::move(j));
        pending.pop_front();
    }
    if (adm.empty()) return PSL_OK;
    const size_t need = adm.size() * (sizeof(WalkDev) + sizeof(BatchEntry) + 2 * sizeof(uint32_t)) + 192;
    if ((size_t)(stage_end - sp) < need) {
        // put them back in order; admitted next iteration
        for (auto it = adm.rbegin(); it != adm.rend(); ++it) {
            const size_t cls = slab_class(slab_layout(it->cfg.L).slab_bytes);
            to_free.emplace(cls, it->slab);
            to_free_bytes += cls;
            used -= it->foot;
            bounds -= it->bound;
            it->slab = nullptr;
            pending.push_front(std::move(*it));
        }
        return PSL_OK;
    }
    // On failure the taken jobs join the active set with whatever slab and
    // slot they hold, so the caller's fail_all releases those and finishes
    // every ticket with the error instead of losing them.
    st = admit_start(adm, sp, stage_end);
    for (auto &j : adm) active.push_back(std::move(j));
    if (st != PSL_OK) return st;
    dirty = true;
    {
        std::lock_guard<std::mutex> g(mu);
        stats.peak_active = std::max<uint64_t>(stats.peak_active, active.size());
        stats.peak_used = std::max<uint64_t>(stats.peak_used, used);
    }
    return PSL_OK;
}

// The fallible part of an admission: slots, walk records, init launches.
psl_status Server::admit_start(std::vector<Job> &adm, char *&sp, char *stage_end)
{
    (void)stage_end;
    if (ctx->test_fail_admit && ++n_admissions == ctx->test_fail_admit)
        return fail(ctx, PSL_E_HIP, "admission %u failed by the test hook", n_admissions);
    psl_status st;
    size_t n_suf = 0;
    for (const Job &j : adm) n_suf += suffix_len(j.cfg.L);
    if ((st = size_bufs({buf(d_admit, adm.size()), buf(d_want, adm.size()), buf(d_adm_s0, n_suf),
                         buf(d_adm_m0, n_suf), buf(d_adm_seg, adm.size() + 1)})))
        return st;
    size_t os = 0;
    uint32_t maxL = 0, maxnw = 0;
    BatchEntry *be = (BatchEntry *)sp;
    sp += sizeof(BatchEntry) * adm.size();
    uint32_t *want = (uint32_t *)sp;
    sp += sizeof(uint32_t) * adm.size();
    uint32_t *adm_off = (uint32_t *)sp;
    sp += sizeof(uint32_t) * (adm.size() + 1);
    sp = (char *)(((uintptr_t)sp + 63) & ~(uintptr_t)63);
    SegMap adm_map{};
    {
        std::vector<uint32_t> aL(adm.size());
        for (size_t b = 0; b < adm.size(); ++b) aL[b] = adm[b].cfg.L;
        adm_map = seg_prefix(aL.data(), (uint32_t)adm.size(), adm_off);
        adm_map.off = d_adm_seg.p;
    }
    const uint64_t t = now_ns();
    for (size_t b = 0; b < adm.size(); ++b) {
        Job &j = adm[b];
        if (ctx->free_slots.empty() && ctx->walks.size() >= ctx->walk_cap)
            return fail(ctx, PSL_E_STATE, "walk capacity exceeded");
        uint32_t slot;
        if (!ctx->free_slots.empty()) {
            slot = ctx->free_slots.back();
            ctx->free_slots.pop_back();
        } else {
            slot = (uint32_t)ctx->walks.size();
            ctx->walks.push_back(WalkHost());
        }
        j.slot = slot;
        const SlabLayout lay = slab_layout(j.cfg.L);
        WalkHost &h = ctx->walks[slot];
        h.active = true;
        h.L = j.cfg.L;
        h.nw = (j.cfg.L + 63) / 64;
        h.n_lmt = j.cfg.n_lmt ? j.cfg.n_lmt : j.cfg.L;
        h.slab = j.slab;
        h.slab_bytes = lay.slab_bytes;
        WalkDev *wd = (WalkDev *)sp;
        sp += sizeof(WalkDev);
        fill_walk(*wd, j.cfg, j.cfg.seed, j.slab, lay);
        j.dev = *wd;
        HIP_TRY(ctx, hipMemsetAsync(j.slab, 0, lay.slab_bytes, ctx->stream));
        HIP_TRY(ctx, hipMemcpyAsync(ctx->d_walks + slot, wd, sizeof(WalkDev), hipMemcpyHostToDevice,
                                    ctx->stream));
        memset(&be[b], 0, sizeof(BatchEntry));
        be[b].slot = slot;
        be[b].S0 = d_adm_s0.p + os;
        be[b].M0 = d_adm_m0.p + os;
        os += suffix_len(j.cfg.L);
        want[b] = 1;
        maxL = std::max(maxL, j.cfg.L);
        maxnw = std::max(maxnw, h.nw);
        j.t_admit = t;
    }
    const uint32_t n = (uint32_t)adm.size();
    HIP_TRY(ctx, hipMemcpyAsync(d_admit.p, be, sizeof(BatchEntry) * n, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(d_want.p, want, sizeof(uint32_t) * n, hipMemcpyHostToDevice, ctx->stream));
    const Tables tabs = tables_of(ctx);
    HIP_TRY(ctx, launch_init_bits(ctx->d_walks, d_admit.p, d_want.p, n, maxnw, ctx->stream));
    HIP_TRY(ctx, launch_corr(ctx->d_walks, d_admit.p, n, maxL, 0, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(d_adm_seg.p, adm_off, sizeof(uint32_t) * (n + 1), hipMemcpyHostToDevice,
                                ctx->stream));
    HIP_TRY(ctx, launch_suffix(ctx->d_walks, d_admit.p, n, maxL, tabs, 2, &adm_map, nullptr, 0, ctx->stream));
    return PSL_OK;
}

// Lays out the admitted batch: entries, eval work items and scratch.
psl_status Server::upload_layout(char *&sp, char *stage_end)
{
    const uint32_t n = (uint32_t)active.size();
    std::vector<uint32_t> Ls(n), nls(n);
    max_L = 0;
    for (uint32_t b = 0; b < n; ++b) {
        Ls[b] = active[b].cfg.L;
        nls[b] = active[b].cfg.n_lmt ? active[b].cfg.n_lmt : active[b].cfg.L;
        max_L = std::max(max_L, Ls[b]);
    }
    EvalLayout lay;
    eval_layout(Ls.data(), nls.data(), n, pick_shape(ctx, Ls.data(), nls.data(), n),
                items_for(ctx, Ls.data(), nls.data(), n), lay);
    const std::vector<uint32_t> &tiles = lay.tiles, &ks = lay.ks;
    size_t n_part = 0, n_cand = 0, n_suf = 0;
    for (uint32_t b = 0; b < n; ++b) {
        n_part += (size_t)ks[b] * nls[b];
        n_cand += nls[b];
        n_suf += suffix_len(Ls[b]);
    }
    const size_t items = lay.items.size();
    shape = lay.shape;
    comb_blocks = lay.comb_blocks;
    comb_group = lay.comb_group;
    const size_t need = sizeof(BatchEntry) * n + sizeof(EvalItem) * items + sizeof(EvalQueues) +
                        sizeof(uint32_t) * (n + 1) + 512;
    if ((size_t)(stage_end - sp) < need) return fail(ctx, PSL_E_NOMEM, "serving staging too small");
    std::vector<uint32_t> off_host(n + 1);
    const SegMap seg_host = seg_prefix(Ls.data(), n, off_host.data());
    // the batch's buffers; the admission buffers may shrink to their least
    psl_status st;
    if ((st = size_bufs({buf(d_batch, n), buf(d_items, items), buf(d_fpart, n_part), buf(d_mpart, n_part),
                         buf(d_f, n_cand), buf(d_p, n_cand), buf(d_s0, n_suf), buf(d_m0, n_suf),
                         buf(d_near, (size_t)(kNearCap + 1) * n), buf(d_queues, 1),
                         buf(d_red, (size_t)comb_blocks * n), buf(d_pend, (size_t)n + 1), buf(d_done, n),
                         buf(d_seg, (size_t)n + 1), buf(d_segtot, seg_host.total),
                         buf(d_segmax, seg_host.total), buf(d_admit, 0), buf(d_want, 0), buf(d_adm_s0, 0),
                         buf(d_adm_m0, 0), buf(d_adm_seg, 0)})))
        return st;
    BatchEntry *be = (BatchEntry *)sp;
    sp += sizeof(BatchEntry) * n;
    sp = (char *)(((uintptr_t)sp + 15) & ~(uintptr_t)15);
    EvalItem *it = (EvalItem *)sp;
    sp += sizeof(EvalItem) * items;
    sp = (char *)(((uintptr_t)sp + 63) & ~(uintptr_t)63);
    size_t op = 0, oc = 0, os = 0;
    for (uint32_t b = 0; b < n; ++b) {
        const Job &j = active[b];
        const uint32_t nl = j.cfg.n_lmt ? j.cfg.n_lmt : j.cfg.L;
        BatchEntry &e = be[b];
        memset(&e, 0, sizeof e);
        e.Fpart = d_fpart.p + op;
        e.Mpart = d_mpart.p + op;
        e.F = d_f.p + oc;
        e.P = d_p.p + oc;
        e.S0 = d_s0.p + os;
        e.M0 = d_m0.p + os;
        e.near = d_near.p + (size_t)(kNearCap + 1) * b;
        e.red = d_red.p + (size_t)comb_blocks * b;
        e.slot = j.slot;
        e.ksplit = ks[b];
        e.tiles = tiles[b];
        e.n_lmt = nl;
        e.near_lim = near_limit_for(ctx, j.cfg.L);
        op += (size_t)ks[b] * nl;
        oc += nl;
        os += suffix_len(j.cfg.L);
    }
    memcpy(it, lay.items.data(), sizeof(EvalItem) * items);
    HIP_TRY(ctx, hipMemcpyAsync(d_batch.p, be, sizeof(BatchEntry) * n, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(d_items.p, it, sizeof(EvalItem) * items, hipMemcpyHostToDevice,
                                ctx->stream));
    EvalQueues *qs = (EvalQueues *)sp;
    sp += sizeof(EvalQueues);
    *qs = lay.queues;
    HIP_TRY(ctx, hipMemcpyAsync(d_queues.p, qs, sizeof(EvalQueues), hipMemcpyHostToDevice, ctx->stream));
    sp = (char *)(((uintptr_t)sp + 63) & ~(uintptr_t)63);
    uint32_t *off = (uint32_t *)sp;
    sp += sizeof(uint32_t) * (n + 1);
    seg = seg_prefix(Ls.data(), n, off);
    seg.off = d_seg.p;
    seg.tot = d_segtot.p;
    seg.tmax = d_segmax.p;
    HIP_TRY(ctx, hipMemcpyAsync(d_seg.p, off, sizeof(uint32_t) * (n + 1), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, launch_near_reset(d_batch.p, n, d_pend.p, d_done.p, ctx->stream));
    n_items = (uint32_t)items;
    dirty = false;
    return PSL_OK;
}

// Both staging halves hold at least `need` bytes (growing waits for the
// stream, so no copy still reads the old buffers).
psl_status Server::ensure_stage(size_t need)
{
    if (need <= stage_cap[0] && need <= stage_cap[1]) return PSL_OK;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const size_t bytes = need + need / 2;
    for (int h = 0; h < 2; ++h) {
        if (stage[h]) (void)hipHostFree(stage[h]);
        stage[h] = nullptr;
        stage_cap[h] = 0;
        stage_used[h] = false;
        HIP_TRY(ctx, hipHostMalloc((void **)&stage[h], bytes, hipHostMallocDefault));
        stage_cap[h] = bytes;
    }
    return PSL_OK;
}

psl_status Server::iterate()
{
    psl_status st;
    // staging half of this iteration: wait for its use two iterations back
    if (stage_used[cur]) {
        HIP_TRY(ctx, hipEventSynchronize(stage_ev[cur]));
        stage_used[cur] = false;
    }
    retire_finished();
    // the slab pool is freed when it grows large (freeing waits for the stream)
    if ((to_free.size() >= kFlushSlabs || to_free_bytes >= kFlushBytes) && (st = flush_free())) return st;
    {
        // worst case of this iteration's uploads: admissions, then the layout
        // (work items <= 8 x (eval_items + candidate tiles) with padding, see eval_layout)
        const size_t n_adm = std::min<size_t>(pending.size(), cfg.max_slots);
        uint64_t tiles = 0;
        const uint32_t tl = 64 * kEvalWavesSmall;
        for (auto &j : active) tiles += ((j.cfg.n_lmt ? j.cfg.n_lmt : j.cfg.L) + tl - 1) / tl;
        for (size_t x = 0; x < n_adm; ++x) {
            const Job &j = pending[x];
            tiles += ((j.cfg.n_lmt ? j.cfg.n_lmt : j.cfg.L) + tl - 1) / tl;
        }
        const size_t need = (n_adm + active.size()) * (sizeof(WalkDev) + 2 * sizeof(BatchEntry) + 16) +
                            sizeof(EvalItem) * 8 * ((uint64_t)items_max(ctx) + tiles) + 8192;
        if ((st = ensure_stage(need))) return st;
    }
    char *sp = stage[cur];
    char *se = stage[cur] + stage_cap[cur];
    if ((st = admit(sp, se))) return st;
    if (active.empty()) return PSL_OK;
    if (dirty && (st = upload_layout(sp, se))) return st;
    const uint32_t n = (uint32_t)active.size();
    const Tables tabs = tables_of(ctx);
    HIP_TRY(ctx, launch_suffix(ctx->d_walks, d_batch.p, n, max_L, tabs, 0, &seg, d_pend.p, shape.waves >= kEvalWavesMax,
                               ctx->stream));
    HIP_TRY(ctx, launch_eval(ctx->d_walks, d_batch.p, d_items.p, n_items, tabs, shape, d_queues.p, ctx->stream));
    HIP_TRY(ctx, launch_select(ctx->d_walks, d_batch.p, n, comb_blocks, comb_group, tabs, 0, nullptr, d_pend.p,
                               d_done.p, ctx->amb_margin, ctx->stream));
    HIP_TRY(ctx, launch_apply(ctx->d_walks, d_batch.p, seg, -1, ctx->stream));
    bool big = false;
    uint64_t units = 0;
    for (auto &j : active) {
        big |= j.cfg.flip_lmt > kFlipIncremental;
        units += pending_units(j.cfg.L);
    }
    if (big) HIP_TRY(ctx, launch_corr(ctx->d_walks, d_batch.p, n, max_L, 1, ctx->stream));
    HIP_TRY(ctx, launch_pending(ctx->d_walks, d_batch.p, n, units, tabs, d_pend.p, ctx->stream));
    uint64_t evals = 0, upd = 0;
    for (auto &j : active) {
        const uint64_t nl = j.cfg.n_lmt ? j.cfg.n_lmt : j.cfg.L;
        evals += nl;
        upd += nl * (j.cfg.L - 1);
        j.steps++;
    }
    // retire walks that reached their budget
    for (size_t x = 0; x < active.size();) {
        Job &j = active[x];
        if (j.steps < j.budget) {
            ++x;
            continue;
        }
        const size_t bytes = sizeof(WalkDev) + 8ull * ((j.cfg.L + 63) / 64);
        if ((st = pinned(ctx, *this, bytes, &j.host))) return st;
        j.host_bytes = bytes;
        HIP_TRY(ctx, hipMemcpyAsync(j.host, ctx->d_walks + j.slot, sizeof(WalkDev), hipMemcpyDeviceToHost,
                                    ctx->stream));
        HIP_TRY(ctx, hipMemcpyAsync(j.host + sizeof(WalkDev), j.dev.best, 8ull * ((j.cfg.L + 63) / 64),
                                    hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(ctx, hipEventCreateWithFlags(&j.ev, hipEventDisableTiming));
        HIP_TRY(ctx, hipEventRecord(j.ev, ctx->stream));
        const size_t cls = slab_class(slab_layout(j.cfg.L).slab_bytes);
        to_free.emplace(cls, j.slab);
        to_free_bytes += cls;
        used -= j.foot;
        bounds -= j.bound;
        j.slab = nullptr;
        ctx->walks[j.slot] = WalkHost();
        ctx->free_slots.push_back(j.slot);
        retiring.push_back(std::move(j));
        active.erase(active.begin() + x);
        dirty = true;
    }
    HIP_TRY(ctx, hipEventRecord(stage_ev[cur], ctx->stream));
    stage_used[cur] = true;
    cur ^= 1;
    std::lock_guard<std::mutex> g(mu);
    stats.iterations++;
    stats.flip_evals += evals;
    stats.ck_updates += upd;
    return PSL_OK;
}

void Server::run()
{
    (void)hipSetDevice(ctx->device);
    for (;;) {
        bool idle;
        {
            std::unique_lock<std::mutex> g(mu);
            while (!incoming.empty()) {
                pending.push_back(std::move(incoming.front()));
                incoming.pop_front();
            }
            if (stop && !drain) break;
            idle = pending.empty() && active.empty();
            if (stop && idle && retiring.empty()) break;
            if (idle && retiring.empty()) {
                if (busy_from) {
                    stats.busy_s += (now_ns() - busy_from) * 1e-9;
                    busy_from = 0;
                }
                cv.wait_for(g, std::chrono::milliseconds(2));
                continue;
            }
            if (!idle && !busy_from) busy_from = now_ns();
            stats.active = active.size();
            stats.queued = pending.size();
        }
        if (idle) {
            // only read-backs in flight
            retire_finished();
            std::this_thread::sleep_for(std::chrono::microseconds(200));
            continue;
        }
        if (iterate() != PSL_OK) fail_all(PSL_E_HIP);
    }
    // cancel what is left (drain == 0) and settle read-backs
    (void)hipStreamSynchronize(ctx->stream);
    retire_finished();
    for (auto &j : retiring) finish(j, PSL_OK);
    retiring.clear();
    for (auto &j : active) {
        dev_free(ctx, j.slab, false);
        j.slab = nullptr;
        ctx->walks[j.slot] = WalkHost();
        ctx->free_slots.push_back(j.slot);
        finish(j, PSL_E_STATE);
    }
    active.clear();
    used = 0;
    bounds = 0;
    (void)flush_free();
    (void)release_scratch();          // a stopped loop holds no device memory
    for (auto &j : pending) finish(j, PSL_E_STATE);
    pending.clear();
    std::lock_guard<std::mutex> g(mu);
    if (busy_from) stats.busy_s += (now_ns() - busy_from) * 1e-9;
    busy_from = 0;
    stats.active = stats.queued = 0;
    running = false;
}

bool serve_active(psl_ctx *ctx)
{
    Server *s = ctx->server;
    if (!s) return false;
    std::lock_guard<std::mutex> g(s->mu);
    return s->running;
}

void serve_shutdown(psl_ctx *ctx)
{
    Server *s = ctx->server;
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->drain = false;
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    (void)hipStreamSynchronize(ctx->stream);
    release(ctx, s->d_batch);
    release(ctx, s->d_admit);
    release(ctx, s->d_items);
    release(ctx, s->d_fpart);
    release(ctx, s->d_f);
    release(ctx, s->d_s0);
    release(ctx, s->d_mpart);
    release(ctx, s->d_m0);
    release(ctx, s->d_near);
    release(ctx, s->d_red);
    release(ctx, s->d_pend);
    release(ctx, s->d_done);
    release(ctx, s->d_seg);
    release(ctx, s->d_adm_seg);
    release(ctx, s->d_segtot);
    release(ctx, s->d_segmax);
    release(ctx, s->d_adm_s0);
    release(ctx, s->d_adm_m0);
    release(ctx, s->d_want);
    release(ctx, s->d_p);
    release(ctx, s->d_queues);
    for (int h = 0; h < 2; ++h) {
        if (s->stage[h]) (void)hipHostFree(s->stage[h]);
        if (s->stage_ev[h]) (void)hipEventDestroy(s->stage_ev[h]);
    }
    for (auto &kv : s->pinned_free) (void)hipHostFree(kv.second);
    delete s;
    ctx->server = nullptr;
}

}  // namespace psl_rt

using namespace psl_rt;

extern "C" {

psl_status psl_serve_start(psl_ctx *ctx, const psl_serve_cfg *cfg)
{
    if (!ctx || !cfg) return PSL_E_INVAL;
    if (cfg->max_slots < 1 || cfg->hbm_budget < 4096 || cfg->flags != 0)
        return fail(ctx, PSL_E_INVAL, "serve cfg: max_slots=%u hbm_budget=%llu", cfg->max_slots,
                    (unsigned long long)cfg->hbm_budget);
    if (ctx->server) {
        bool running;
        {
            std::lock_guard<std::mutex> g(ctx->server->mu);
            running = ctx->server->running;
        }
        if (running) return fail(ctx, PSL_E_STATE, "already serving");
        serve_shutdown(ctx);   // a stopped loop: drop its results
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    psl_status st;
    if ((st = ensure_tables(ctx, PSL_L_MAX))) return st;
    if ((st = ensure_walk_cap(ctx, (uint32_t)ctx->walks.size() + cfg->max_slots))) return st;
    Server *s = new Server();
    s->cfg = *cfg;
    s->ctx = ctx;
    s->items_cap = items_max(ctx);
    {
        // the budget has to fit the device's free memory (taken as jobs come)
        size_t dfree = 0, dtotal = 0;
        if (hipMemGetInfo(&dfree, &dtotal) != hipSuccess || dfree < cfg->hbm_budget) {
            (void)hipGetLastError();
            delete s;
            return fail(ctx, PSL_E_NOMEM, "hbm_budget of %llu bytes exceeds the free device memory (%zu)",
                        (unsigned long long)cfg->hbm_budget, dfree);
        }
    }
    const size_t stage_bytes = ((size_t)4 << 20) + (size_t)cfg->max_slots * 256;
    for (int h = 0; h < 2; ++h) {
        if (hipHostMalloc((void **)&s->stage[h], stage_bytes, hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&s->stage_ev[h], hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            ctx->server = s;
            serve_shutdown(ctx);
            return fail(ctx, PSL_E_HIP, "serving staging");
        }
        s->stage_cap[h] = stage_bytes;
    }
    s->running = true;
    ctx->server = s;
    s->th = std::thread([s] { s->run(); });
    return PSL_OK;
}

psl_status psl_serve_submit(psl_ctx *ctx, const psl_job *job, uint64_t *ticket)
{
    if (!ctx || !job || !ticket) return PSL_E_INVAL;
    Server *s = ctx->server;
    if (!s) return PSL_E_STATE;
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (!s->running || s->stop) return PSL_E_STATE;
    }
    const psl_walk_cfg &c = job->cfg;
    if (c.L < 2 || c.L > PSL_L_MAX || c.alpha1 < 1 || c.alpha1 > PSL_ALPHA_MAX || c.alpha2 < 1 ||
        c.alpha2 > PSL_ALPHA_MAX || c.n_lmt > c.L || c.flip_lmt > c.L || c.flip_lmt > PSL_FLIP_LMT_MAX ||
        c.reserved != 0 || job->step_budget < 1)
        return PSL_E_INVAL;
    Job j;
    j.cfg = c;
    j.budget = job->step_budget;
    j.best_out = job->best_bits_out;
    j.t_arrive = now_ns();
    j.bound = scratch_bound(c.L, c.n_lmt ? c.n_lmt : c.L, s->items_cap);
    j.foot = slab_class(slab_layout(c.L).slab_bytes) + j.bound;
    if (j.foot > s->cfg.hbm_budget) return PSL_E_FULL;
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (!s->running || s->stop) return PSL_E_STATE;
        j.ticket = s->next_ticket++;
        *ticket = j.ticket;
        s->live[j.ticket] = 1;
        s->incoming.push_back(std::move(j));
        s->stats.submitted++;
    }
    s->cv.notify_one();
    return PSL_OK;
}

psl_status psl_serve_poll(psl_ctx *ctx, uint64_t ticket, psl_job_result *out)
{
    if (!ctx || !out) return PSL_E_INVAL;
    Server *s = ctx->server;
    if (!s) return PSL_E_STATE;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->done.find(ticket);
    if (it != s->done.end()) {
        *out = it->second;
        s->done.erase(it);
        return PSL_OK;
    }
    return s->live.count(ticket) ? PSL_E_AGAIN : PSL_E_STATE;
}

psl_status psl_serve_footprint(const psl_walk_cfg *cfg, uint64_t *bytes)
{
    if (!cfg || !bytes || cfg->L < 2 || cfg->L > PSL_L_MAX || cfg->n_lmt > cfg->L) return PSL_E_INVAL;
    *bytes = job_footprint(*cfg, kEvalItemsDefault);
    return PSL_OK;
}

psl_status psl_serve_stats_read(psl_ctx *ctx, psl_serve_stats *out)
{
    if (!ctx || !out) return PSL_E_INVAL;
    Server *s = ctx->server;
    if (!s) return PSL_E_STATE;
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    if (s->busy_from) out->busy_s += (now_ns() - s->busy_from) * 1e-9;
    return PSL_OK;
}

psl_status psl_serve_stop(psl_ctx *ctx, int drain)
{
    if (!ctx) return PSL_E_INVAL;
    Server *s = ctx->server;
    if (!s) return PSL_E_STATE;
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (!s->running && !s->th.joinable()) return PSL_OK;
        s->stop = true;
        s->drain = drain != 0;
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    return PSL_OK;
}

}  // extern "C"
