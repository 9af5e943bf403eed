// psl_kernels.hip -- gfx950 kernels of libpsl around the neighbourhood
// evaluation (which lives in psl_eval.hip): power tables, init and the
// correlations of Eq. (2), the phase-switch rebuild, the per-step chunk sums
// and near-peak list the evaluation reads, the selection of Algorithm 1's
// scan, the O(L) flip of Section 3 and the step's bookkeeping.
#include "psl_dev_util.h"
#include "psl_device.h"
#include "psl_launch.h"

#include <algorithm>
#include <climits>

namespace psl {

// ------------------------------------------------------- power tables

__global__ void k_power_table(double *T, uint32_t n, uint32_t alpha)
{
    uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double x = (double)c, p = x;
    for (uint32_t a = 1; a < alpha; ++a) p = p * x;
    T[c] = p;
}

// ------------------------------------------------------------- init

// Random initial pivots (Rand(L, SEED)) for batch entries with want[b] != 0,
// then local_best = best = pivot for every entry.
__global__ void k_init_bits(WalkDev *walks, const BatchEntry *batch, const uint32_t *want)
{
    WalkDev &w = walks[batch[blockIdx.y].slot];
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= w.nw) return;
    uint64_t v = w.pivot[i];
    if (want[blockIdx.y]) {
        v = draw(w.seed, i);
        if (i == w.nw - 1 && (w.L & 63u)) v &= (1ull << (w.L & 63u)) - 1ull;
        w.pivot[i] = v;
    }
    w.local_best[i] = v;
    w.best[i] = v;
}

// Eq. (2) from the packed pivot: C_k = (L-k) - 2 * #(s_i != s_{i+k}).
// A block owns 256 consecutive shifts k0..k0+255 and sweeps the sequence in
// LDS-staged segments of 32-bit words: word x of the sequence and the word at
// bit offset 32x + k (one funnel shift of two staged words) give 32 products
// per XOR and popcount.
// only_pending == 0: every walk (init; C of local_best = C as well);
// only_pending == 1: walks left pending by a switch whose Rand_flip is too
// large for the one-flip rebuild (k_switch_corr);
// only_pending == 2: every walk, C only (checkpoint restore).
constexpr int kCorrThreads = 256;
constexpr int kCorrSeg = 1024;        // staged 32-bit words per segment
__global__ __launch_bounds__(kCorrThreads) void k_corr(WalkDev *walks, const BatchEntry *batch,
                                                       int only_pending)
{
    WalkDev &w = walks[batch[blockIdx.y].slot];
    if (only_pending == 1 && !(w.pending && w.n_flips > kFlipIncremental)) return;
    const uint32_t L = w.L;
    const uint32_t k0 = blockIdx.x * kCorrThreads;
    if (k0 >= L) return;
    __shared__ uint32_t A[kCorrSeg];
    __shared__ uint32_t B[kCorrSeg + 16];
    const uint32_t *s32 = reinterpret_cast<const uint32_t *>(w.pivot);
    const uint32_t n32 = (L + 31) / 32;
    const uint32_t k = k0 + threadIdx.x;
    const uint32_t d = threadIdx.x, dq = d >> 5, dr = d & 31u;
    const uint32_t nprod = k < L ? L - k : 0;          // products of this shift
    const uint32_t nwb = (L - k0 + 31) / 32;           // words the block needs
    const uint32_t kq = k0 / 32;
    uint32_t diff = 0;
    for (uint32_t w0 = 0; w0 < nwb; w0 += kCorrSeg) {
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < kCorrSeg; t += kCorrThreads)
            A[t] = (w0 + t < n32) ? s32[w0 + t] : 0u;
        for (uint32_t t = threadIdx.x; t < kCorrSeg + 16; t += kCorrThreads)
            B[t] = (w0 + kq + t < n32) ? s32[w0 + kq + t] : 0u;
        __syncthreads();
        // this shift's products in the segment: bits 32*w0 .. nprod
        const uint32_t have = nprod > 32 * w0 ? nprod - 32 * w0 : 0;
        const uint32_t full = min((uint32_t)kCorrSeg, have / 32);
        for (uint32_t x = 0; x < full; ++x)
            diff += __popc(A[x] ^ __builtin_amdgcn_alignbit(B[x + dq + 1], B[x + dq], dr));
        if (full < (uint32_t)kCorrSeg && (have & 31u)) {
            const uint32_t x = full;
            const uint32_t v = A[x] ^ __builtin_amdgcn_alignbit(B[x + dq + 1], B[x + dq], dr);
            diff += __popc(v & ((1u << (have & 31u)) - 1u));
        }
    }
    if (k < L) {
        const int32_t c = (int32_t)nprod - 2 * (int32_t)diff;
        w.C[k] = c;
        if (only_pending == 0) w.C_lb[k] = c;
    }
}

// The pending list of a batch: pend[0] = count, pend[1..] = batch positions
// of the walks whose step ended in a phase switch (the bookkeeping appends,
// the selection of the next step clears the count).
//
// C of a switched pivot from C of local_best: the FLIP_lmt one-element flips
// in draw order, where flip f sees local_best with flips 0..f-1 applied.
// Element x of that sequence differs from local_best only if x is an earlier
// flip position, and flip f reads elements p_f and p_f +- k; so for every k
// outside D = {|p_f - p_g| : g < f} the update can read local_best's bits
// directly, and the shifts in D take the sequential bits.
__device__ __forceinline__ int32_t switch_flip_delta(const uint64_t *lb, uint32_t L, uint32_t k, uint32_t p)
{
    const int sp = get_bit(lb, p) ? -1 : 1;
    int d = 0;
    if (p + k < L) d += get_bit(lb, p + k) ? -1 : 1;
    if (k <= p) d += get_bit(lb, p - k) ? -1 : 1;
    return -2 * sp * d;
}

// C_k of the switched pivot for a shift k in D: each flip reads the elements
// as the earlier flips left them.
__device__ __forceinline__ int32_t switch_corr_seq(const uint64_t *lb, const int32_t *C_lb, uint32_t L,
                                                   uint32_t k, const uint32_t *fl, uint32_t nf)
{
    int32_t c = C_lb[k];
    for (uint32_t h = 0; h < nf; ++h) {
        // element x after flips 0..h-1
        auto bit = [&](uint32_t x) {
            uint32_t v = get_bit(lb, x);
            for (uint32_t e = 0; e < h; ++e) v ^= (fl[e] == x) ? 1u : 0u;
            return v;
        };
        const uint32_t p = fl[h];
        const int sp = bit(p) ? -1 : 1;
        int d = 0;
        if (p + k < L) d += bit(p + k) ? -1 : 1;
        if (k <= p) d += bit(p - k) ? -1 : 1;
        c -= 2 * sp * d;
    }
    return c;
}

// After the step's bookkeeping, in two launches: C of every pending walk's
// new pivot from C of its local best (a switch of more than kFlipIncremental
// flips has C rebuilt by k_corr before), then F (Eq. (5)) and the PSL (Eq.
// (3)) of that pivot, which become F_pivot, psl_pivot and v_local.
// k_pending: work units of kPendUnit shifts are dealt round-robin over the
// grid, walk after walk. A unit marks the shifts of D in its range in an LDS
// bitmap, computes and stores its C values, and leaves the sum of T(|C_k|)
// (lanes, then wavefronts, in a fixed order) and the maximum |C_k| in the
// walk's chunk arrays. k_pending_fin adds each walk's unit sums in unit order.
constexpr int kPendThreads = 256;

__global__ __launch_bounds__(kPendThreads) void k_pending(WalkDev *walks, const BatchEntry *batch, Tables tabs,
                                                          const uint32_t *pend)
{
    __shared__ uint32_t s_fl[kFlipIncremental];
    __shared__ uint32_t s_in[kPendUnit / 32];
    __shared__ double s_s[kPendThreads / 64], s_c[kPendThreads / 64];
    __shared__ uint32_t s_m[kPendThreads / 64];
    const uint32_t np = pend[0];
    const uint32_t G = gridDim.x;
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    uint32_t base = 0;                  // units of the earlier pending walks
    for (uint32_t q = 0; q < np; ++q) {
        const BatchEntry be = batch[pend[1 + q]];
        WalkDev &w = walks[be.slot];
        const uint32_t L = w.L;
        const uint32_t nu = (L - 1 + kPendUnit - 1) / kPendUnit;
        const uint32_t nf = w.n_flips;
        const bool incr = nf <= kFlipIncremental;
        const double *T = tabs.T[w.alpha];
        for (uint32_t u = (blockIdx.x + G - base % G) % G; u < nu; u += G) {
            const uint32_t k_lo = 1 + u * kPendUnit, k_hi = min(L, k_lo + kPendUnit);
            __syncthreads();            // the previous unit is done with the LDS
            if (incr) {
                if (threadIdx.x < nf) s_fl[threadIdx.x] = w.flips[threadIdx.x];
                if (threadIdx.x < kPendUnit / 32) s_in[threadIdx.x] = 0;
            }
            __syncthreads();
            if (incr) {
                for (uint32_t pr = threadIdx.x; pr < nf * nf; pr += kPendThreads) {
                    const uint32_t f = pr / nf, g = pr - f * nf;
                    if (g >= f) continue;
                    const uint32_t k = s_fl[f] > s_fl[g] ? s_fl[f] - s_fl[g] : s_fl[g] - s_fl[f];
                    if (k >= k_lo && k < k_hi) atomicOr(&s_in[(k - k_lo) >> 5], 1u << ((k - k_lo) & 31u));
                }
            }
            __syncthreads();
            double ts = 0.0, tc = 0.0;
            uint32_t tm = 0;
            for (uint32_t k = k_lo + threadIdx.x; k < k_hi; k += kPendThreads) {
                int32_t c;
                if (incr) {
                    const uint32_t o = k - k_lo;
                    if ((s_in[o >> 5] >> (o & 31u)) & 1u) {
                        c = switch_corr_seq(w.local_best, w.C_lb, L, k, s_fl, nf);
                    } else {
                        c = w.C_lb[k];
                        for (uint32_t f = 0; f < nf; ++f) c += switch_flip_delta(w.local_best, L, k, s_fl[f]);
                    }
                    w.C[k] = c;
                } else {
                    c = w.C[k];
                }
                const uint32_t a = (uint32_t)(c < 0 ? -c : c);
                nsum_add(ts, tc, T[a]);
                tm = max(tm, a);
            }
            // every lane of the butterfly ends with the same sums
            for (int o = 32; o > 0; o >>= 1) {
                const double ps = __shfl_xor(ts, o), pc = __shfl_xor(tc, o);
                const uint32_t pm = (uint32_t)__shfl_xor((int)tm, o);
                nsum_add(ts, tc, ps);
                tc += pc;
                tm = max(tm, pm);
            }
            if (lane == 0) {
                s_s[wave] = ts;
                s_c[wave] = tc;
                s_m[wave] = tm;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                double us = 0.0, uc = 0.0;
                uint32_t um = 0;
                for (int x = 0; x < kPendThreads / 64; ++x) {
                    nsum_add(us, uc, s_s[x]);
                    uc += s_c[x];
                    um = max(um, s_m[x]);
                }
                be.S0[2 * u] = us;
                be.S0[2 * u + 1] = uc;
                be.M0[u] = um;
            }
        }
        base += nu;
    }
}

// One wavefront per pending walk: the units' sums in unit order.
__global__ __launch_bounds__(64) void k_pending_fin(WalkDev *walks, const BatchEntry *batch, const uint32_t *pend)
{
    const uint32_t np = pend[0];
    const int lane = (int)threadIdx.x;
    for (uint32_t q = blockIdx.x; q < np; q += gridDim.x) {
        const BatchEntry be = batch[pend[1 + q]];
        WalkDev &w = walks[be.slot];
        const uint32_t nu = (w.L - 1 + kPendUnit - 1) / kPendUnit;
        // lane l adds units l, l + 64, ... in order, then the lanes in a
        // fixed butterfly (every lane ends with the same sums)
        double s = 0.0, c = 0.0;
        uint32_t m = 0;
        for (uint32_t x = (uint32_t)lane; x < nu; x += 64) {
            nsum_add(s, c, be.S0[2 * x]);
            c += be.S0[2 * x + 1];
            m = max(m, be.M0[x]);
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ps = __shfl_xor(s, o), pc = __shfl_xor(c, o);
            const uint32_t pm = (uint32_t)__shfl_xor((int)m, o);
            nsum_add(s, c, ps);
            c += pc;
            m = max(m, pm);
        }
        if (lane == 0) {
            const double F = s + c;
            w.F_pivot = F;
            w.psl_pivot = (int32_t)m;
            w.value_local = F;
            w.unimproved = 0;
            w.pending = 0;
        }
    }
}

// F of the pivot (Eq. (5)) and its PSL (Eq. (3)) from C, one block per walk,
// fixed blocking so a given C always gives the same F bits.
// mode 0: initial (value_local, F_pivot, psl_pivot, psl_best);
// mode 2: after a forced flip or a restore (F_pivot, psl_pivot).
constexpr int kFitThreads = 256;
__global__ __launch_bounds__(kFitThreads) void k_fitness(WalkDev *walks, const BatchEntry *batch,
                                                         Tables tabs, int mode)
{
    WalkDev &w = walks[batch[blockIdx.x].slot];
    const double *T = tabs.T[w.alpha];
    double sum = 0.0, comp = 0.0;
    int32_t peak = 0;
    for (uint32_t k = 1 + threadIdx.x; k < w.L; k += kFitThreads) {
        int32_t c = w.C[k];
        int32_t a = c < 0 ? -c : c;
        nsum_add(sum, comp, T[a]);
        peak = a > peak ? a : peak;
    }
    __shared__ double s_sum[kFitThreads], s_comp[kFitThreads];
    __shared__ int32_t s_peak[kFitThreads];
    s_sum[threadIdx.x] = sum;
    s_comp[threadIdx.x] = comp;
    s_peak[threadIdx.x] = peak;
    __syncthreads();
    for (int h = kFitThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            double a = s_sum[threadIdx.x], ca = s_comp[threadIdx.x];
            nsum_add(a, ca, s_sum[threadIdx.x + h]);
            s_sum[threadIdx.x] = a;
            s_comp[threadIdx.x] = ca + s_comp[threadIdx.x + h];
            int32_t p2 = s_peak[threadIdx.x + h];
            if (p2 > s_peak[threadIdx.x]) s_peak[threadIdx.x] = p2;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double F = s_sum[0] + s_comp[0];
        int32_t p = s_peak[0];
        w.F_pivot = F;
        w.psl_pivot = p;
        if (mode == 0) {
            w.value_local = F;
            w.psl_best = p;
        }
    }
}

// --------------------------------------------- neighbourhood evaluation

// Per walk and step, from the pivot's C:
//  * chunk suffix sums S0[x] = sum_{1+32x <= k' < L} T(|C_k'|) and
//    M0[x] = max |C_k'| over the same range, x = 0..nchunks (the last entry
//    0). A candidate j leaves every C_k with k > max(j, L-1-j) unchanged
//    (both neighbours of the flipped element are out of bounds), so that
//    part of its F (and PSL) is read from them; the evaluation only needs
//    them at 32-shift chunk starts;
//  * the near-peak shift list: with P the pivot's PSL, every neighbour has
//    PSL >= P - 4 (one flip moves each C_k by at most 4), and a shift with
//    |C_k| <= P - 9 reaches at most P - 5, so a neighbour's PSL is the maximum
//    of |C'_k| over the shifts with |C_k| >= P - 8 alone. near[0] = count,
//    near[1..] = those shifts (any order), while the count fits kNearCap.
// Two kernels: k_chunks (several blocks per walk) writes per-chunk sums and
// maxima and appends to the near list; k_seg_scan (step) or k_scan (init)
// turns the chunk values into suffix values in a fixed order. The same pair
// is also the fitness of a pivot: S0[0] = F and M0[0] = PSL (mode 2, init).
constexpr int kChunkThreads = 256;
constexpr uint32_t kMaxGridY = 65535;      // walks per launch of the 2-D grids
// Octets o0, o0 + step, ... below o1 of one walk (an octet is 256 consecutive
// shifts, eight chunks), for the calling wavefront: four coalesced passes of
// 64 shifts put T(|C_k|) and |C_k| in the wavefront's LDS rows (sv, sa); then
// lane l adds the four consecutive values 4(l mod 8) .. +3 of chunk l / 8
// (left to right) and a three-level butterfly over the chunk's eight lanes
// finishes its sum and maximum, the same in all eight. The octet's total (a
// fixed tree over its chunks) goes into the wavefront's running total.
__device__ __forceinline__ void chunk_octs(const BatchEntry &be, const WalkDev &w, const double *T, int cut,
                                           bool near, int o0, int o1, int step, double *sv, int *sa,
                                           double &ws, double &wc, uint32_t &wm)
{
    const int L = (int)w.L;
    const int nchunks = (L - 1 + 31) / 32;
    const int lane = threadIdx.x & 63;
    for (int o = o0; o < o1; o += step) {
        // the four passes' C values, then their T values, are all loaded
        // before any is used (two waits per octet, not eight)
        int av[4];
        double tv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 1 + 256 * o + 64 * i + lane;
            const int32_t x = k < L ? w.C[k] : 0;
            av[i] = x < 0 ? -x : x;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 1 + 256 * o + 64 * i + lane;
            tv[i] = k < L ? T[av[i]] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = 64 * i + lane;
            const int k = 1 + 256 * o + e;
            const int a = av[i];
            sv[e] = tv[i];
            sa[e] = a;
            if (near) {
                const bool take = k < L && a >= cut;
                const uint64_t bal = __ballot(take);
                if (bal) {
                    uint32_t base = 0;
                    if (lane == 0) base = atomicAdd(&be.near[0], (uint32_t)__popcll(bal));
                    base = (uint32_t)__shfl((int)base, 0);
                    const uint32_t q = base + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
                    if (take && q < (uint32_t)kNearCap) be.near[1 + q] = (uint32_t)k;
                }
            }
        }
        // the wavefront's rows are written before any lane reads them
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int r = 32 * (lane >> 3) + 4 * (lane & 7);
        double v = sv[r];
        v += sv[r + 1];
        v += sv[r + 2];
        v += sv[r + 3];
        int m = max(max(sa[r], sa[r + 1]), max(sa[r + 2], sa[r + 3]));
        for (int d = 1; d < 8; d <<= 1) {
            v += __shfl_xor(v, d);
            m = max(m, __shfl_xor(m, d));
        }
        const int c = 8 * o + (lane >> 3);
        if ((lane & 7) == 0 && c < nchunks) {
            be.S0[c] = v;
            be.M0[c] = (uint32_t)m;
        }
        // the octet's total over its chunk leaders (every lane ends with it)
        double ts = v, tc = 0.0;
        for (int d = 8; d < 64; d <<= 1) {
            const double ps = __shfl_xor(ts, d), pc = __shfl_xor(tc, d);
            nsum_add(ts, tc, ps);
            tc += pc;
            m = max(m, __shfl_xor(m, d));
        }
        nsum_add(ws, wc, ts);
        wc += tc;
        wm = max(wm, (uint32_t)m);
        // every lane has read the rows before the next octet overwrites them
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// Mode 0 (step, with the near list) and 2 (init): one block per segment of
// the map.
__global__ __launch_bounds__(kChunkThreads) void k_chunks(const WalkDev *walks, const BatchEntry *batch,
                                                          Tables tabs, int mode, SegMap map, uint32_t *pend)
{
    // the previous step's pending list has been consumed; this step's
    // bookkeeping (in the selection) refills it
    if (pend && blockIdx.x == 0 && threadIdx.x == 0) pend[0] = 0;
    const int wave = (int)threadIdx.x >> 6;
    constexpr int kWaves = kChunkThreads / 64;
    uint32_t b, seg;
    seg_of(map, blockIdx.x, b, seg);
    const BatchEntry be = batch[b];
    const WalkDev &w = walks[be.slot];
    const int nocts = ((int)w.L - 1 + 255) / 256;
    const int octs_per_seg = 1 << (map.shift - 8);
    const int o0 = (int)seg * octs_per_seg;
    const int o1 = min(nocts, o0 + octs_per_seg);
    __shared__ double s_v[kWaves][256];
    __shared__ int s_a[kWaves][256];
    // the near-peak cut (the pivot's PSL is kept current by every step)
    double ws = 0.0, wc = 0.0;
    uint32_t wm = 0;
    chunk_octs(be, w, tabs.T[w.alpha], w.psl_pivot - 8, mode == 0, o0 + wave, o1, kWaves, s_v[wave], s_a[wave],
               ws, wc, wm);
    if (map.tot) {
        // the segment's total (waves in order) for the segment-parallel scan
        __shared__ double s_s[kWaves], s_c[kWaves];
        __shared__ uint32_t s_m[kWaves];
        if ((threadIdx.x & 63) == 0) {
            s_s[wave] = ws;
            s_c[wave] = wc;
            s_m[wave] = wm;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double ts = 0.0, tc = 0.0;
            uint32_t tm = 0;
            for (int x = 0; x < kWaves; ++x) {
                nsum_add(ts, tc, s_s[x]);
                tc += s_c[x];
                tm = max(tm, s_m[x]);
            }
            map.tot[blockIdx.x] = ts + tc;
            map.tmax[blockIdx.x] = tm;
        }
    }
}

// Suffix values of the step's chunk arrays, one wavefront per segment of the
// map: the segment's chunks (at most 128, two per lane) are scanned from the
// right with doubling steps, and the offset is the sum of the totals of the
// walk's later segments (a fixed butterfly over lanes). Each entry is a sum
// of the same chunk values, each in a fixed order.
constexpr int kSegScanThreads = 256;
__global__ __launch_bounds__(kSegScanThreads) void k_seg_scan(const WalkDev *walks, const BatchEntry *batch,
                                                              SegMap map)
{
    const uint32_t i = blockIdx.x * (kSegScanThreads / 64) + (threadIdx.x >> 6);
    if (i >= map.total) return;              // wave-uniform
    const int lane = threadIdx.x & 63;
    uint32_t b, seg;
    seg_of(map, i, b, seg);
    const BatchEntry be = batch[b];
    const WalkDev &w = walks[be.slot];
    const int nchunks = ((int)w.L - 1 + 31) / 32;
    const int cps = 1 << (map.shift - 5);    // chunks per segment
    const int c0 = (int)seg * cps;
    const int c1 = min(nchunks, c0 + cps);
    // totals of the later segments of this walk
    const uint32_t last = map.off ? map.off[b + 1] : (b + 1) * map.spw;
    double os = 0.0, oc = 0.0;
    uint32_t om = 0;
    for (uint32_t x = i + 1 + lane; x < last; x += 64) {
        nsum_add(os, oc, map.tot[x]);
        om = max(om, map.tmax[x]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double ps = __shfl_xor(os, o), pc = __shfl_xor(oc, o);
        const uint32_t pm = (uint32_t)__shfl_xor((int)om, o);
        nsum_add(os, oc, ps);
        oc += pc;
        om = max(om, pm);
    }
    // lane l holds chunks c0 + 2l, c0 + 2l + 1
    const int ca = c0 + 2 * lane, cb = ca + 1;
    const double va = ca < c1 ? be.S0[ca] : 0.0, vb = cb < c1 ? be.S0[cb] : 0.0;
    const uint32_t ma = ca < c1 ? be.M0[ca] : 0u, mb = cb < c1 ? be.M0[cb] : 0u;
    double ls = 0.0, lc = 0.0;
    nsum_add(ls, lc, vb);
    nsum_add(ls, lc, va);
    uint32_t lm = max(ma, mb);
    // inclusive suffix over lanes, then exclusive by one lane
    for (int d = 1; d < 64; d <<= 1) {
        const double ps = __shfl_down(ls, d), pc = __shfl_down(lc, d);
        const uint32_t pm = (uint32_t)__shfl_down((int)lm, d);
        if (lane + d < 64) {
            nsum_add(ls, lc, ps);
            lc += pc;
            lm = max(lm, pm);
        }
    }
    double es = __shfl_down(ls, 1), ec = __shfl_down(lc, 1);
    uint32_t em = (uint32_t)__shfl_down((int)lm, 1);
    if (lane == 63) {
        es = 0.0;
        ec = 0.0;
        em = 0;
    }
    // add the later segments, then this lane's chunks from the right
    nsum_add(es, ec, os);
    ec += oc;
    em = max(em, om);
    if (cb < c1) {
        nsum_add(es, ec, vb);
        em = max(em, mb);
        be.S0[cb] = es + ec;
        be.M0[cb] = em;
    }
    if (ca < c1) {
        nsum_add(es, ec, va);
        em = max(em, ma);
        be.S0[ca] = es + ec;
        be.M0[ca] = em;
    }
    if (c1 == nchunks && lane == 0) {
        be.S0[nchunks] = 0.0;
        be.M0[nchunks] = 0;
    }
}

constexpr int kScanThreads = 1024;
// The initial fitness: block b scans walk b's chunk sums into suffix values
// and sets value_local, F_pivot, psl_pivot and psl_best.
__global__ __launch_bounds__(kScanThreads) void k_scan(WalkDev *walks, const BatchEntry *batch)
{
    const BatchEntry be = batch[blockIdx.x];
    WalkDev &w = walks[be.slot];
    const int L = (int)w.L;
    const int nchunks = (L - 1 + 31) / 32;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ double s_ts[kScanThreads], s_tc[kScanThreads];
    __shared__ uint32_t s_tm[kScanThreads];

    // each thread a contiguous segment (right to left, Neumaier), then an
    // exclusive suffix scan of the segment totals (one wave, 16 per lane),
    // then the offsets
    const int seg = (nchunks + kScanThreads - 1) / kScanThreads;
    const int lo = (int)threadIdx.x * seg, hi = min(nchunks, lo + seg);
    double ts = 0.0, tc = 0.0;
    uint32_t tm = 0;
#pragma unroll 4
    for (int c = hi - 1; c >= lo; --c) {
        nsum_add(ts, tc, be.S0[c]);
        tm = max(tm, be.M0[c]);
    }
    s_ts[threadIdx.x] = ts;
    s_tc[threadIdx.x] = tc;
    s_tm[threadIdx.x] = tm;
    __syncthreads();
    if (wave == 0) {
        // lane l owns segment totals 16l .. 16l+15
        double ls = 0.0, lc = 0.0;
        uint32_t lm = 0;
        for (int x = 15; x >= 0; --x) {
            const int t = 16 * lane + x;
            nsum_add(ls, lc, s_ts[t]);
            lc += s_tc[t];
            lm = max(lm, s_tm[t]);
        }
        // inclusive suffix over lanes in six doubling steps, then shifted
        // down one lane: the totals of the lanes above l
        for (int d = 1; d < 64; d <<= 1) {
            const double os = __shfl_down(ls, d), oc = __shfl_down(lc, d);
            const uint32_t om = (uint32_t)__shfl_down((int)lm, d);
            if (lane + d < 64) {
                nsum_add(ls, lc, os);
                lc += oc;
                lm = max(lm, om);
            }
        }
        double es = __shfl_down(ls, 1), ec = __shfl_down(lc, 1);
        uint32_t em = (uint32_t)__shfl_down((int)lm, 1);
        if (lane == 63) {
            es = 0.0;
            ec = 0.0;
            em = 0;
        }
        for (int x = 15; x >= 0; --x) {
            const int t = 16 * lane + x;
            const double ns = s_ts[t], nc = s_tc[t];
            const uint32_t nm = s_tm[t];
            s_ts[t] = es;
            s_tc[t] = ec;
            s_tm[t] = em;
            nsum_add(es, ec, ns);
            ec += nc;
            em = max(em, nm);
        }
    }
    __syncthreads();
    ts = s_ts[threadIdx.x];
    tc = s_tc[threadIdx.x];
    tm = s_tm[threadIdx.x];
    for (int c = hi - 1; c >= lo; --c) {
        nsum_add(ts, tc, be.S0[c]);
        tm = max(tm, be.M0[c]);
        be.S0[c] = ts + tc;
        be.M0[c] = tm;
    }
    if (threadIdx.x == 0) {
        be.S0[nchunks] = 0.0;
        be.M0[nchunks] = 0;
        // thread 0's segment starts at chunk 0: the totals over k >= 1
        const double F = ts + tc;
        w.F_pivot = F;
        w.psl_pivot = (int32_t)tm;
        w.value_local = F;
        w.psl_best = (int32_t)tm;
    }
}

// ------------------------------------------------------- selection

struct ChoiceDev {
    uint32_t i_best, j_best;
    double F_best, F_min;
    uint32_t j_psl;
    int32_t psl_min;
    int32_t psl_k;
    uint32_t flags;         // CHOICE_AMBIG_ARGMIN (set with the selection)
};

constexpr int kCombThreads = 256;
constexpr int kCombBatch = 16;      // split loads a combine lane keeps in flight
constexpr uint64_t kCombFuseBlocks = 256;   // most combine blocks of a launch that selects in its last blocks

// Candidates [lo, hi) of combine block b of `blocks`: contiguous ranges in
// scan order, a multiple of the block's candidates per pass (kCombThreads / G)
// long, so a block's minimum covers a contiguous run of scan indices.
__device__ __forceinline__ void comb_range(uint32_t n, uint32_t blocks, uint32_t G, uint32_t b, uint32_t &lo,
                                           uint32_t &hi)
{
    const uint32_t cpb = kCombThreads / G;
    const uint32_t chunk = ((n + blocks - 1) / blocks + cpb - 1) / cpb * cpb;
    lo = min(n, b * chunk);
    hi = min(n, lo + chunk);
}

__device__ __forceinline__ void sel_merge(double &f, int32_t &p, uint32_t &i, double of, int32_t op,
                                          uint32_t oi)
{
    f = of < f ? of : f;
    if (op < p || (op == p && oi < i)) {
        p = op;
        i = oi;
    }
}

// The scan of Algorithm 1 over the combined F and PSL: the move is the first
// candidate in scan order within F_min*(1+tau); the best-PSL neighbour is the
// first with the minimum PSL.
// pure != 0: write the choice to out[b] and leave the walk unchanged.
// Otherwise record the choice in the walk and, on a strict PSL improvement,
// update psl_best and solution_best = pivot with j_psl flipped.
// The selection of walk w (batch position bi) by a block of NT threads.
template <int NT>
__device__ __forceinline__ void select_walk(WalkDev &w, const BatchEntry &be, uint32_t bi, uint32_t comb_blocks,
                                            uint32_t comb_group, int pure, ChoiceDev *out)
{
    const uint32_t n = be.fixed ? be.n_lmt : w.n_lmt;
    const uint32_t start = be.fixed ? be.start : step_start(w);
    const uint32_t L = w.L;

    double fmin = INFINITY;
    int32_t pmin = INT_MAX;
    uint32_t ipmin = UINT_MAX;
    if (threadIdx.x < comb_blocks) {
        const SelPart r = be.red[threadIdx.x];
        fmin = r.f;
        pmin = r.p;
        ipmin = r.i;
    }
    const double my_f = fmin;           // this thread's combine block minimum
    // block minima: within each wavefront, then across the wavefronts (the
    // minimum F and the first minimum (PSL, index) do not depend on the order)
    constexpr int kSelWaves = NT / 64;
    __shared__ SelPart s_w[kSelWaves];
    __shared__ uint32_t s_first[kSelWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) {
        const double of = __shfl_xor(fmin, o);
        const int32_t op = __shfl_xor(pmin, o);
        const uint32_t oi = (uint32_t)__shfl_xor((int)ipmin, o);
        sel_merge(fmin, pmin, ipmin, of, op, oi);
    }
    if (lane == 0) s_w[wave] = SelPart{fmin, pmin, ipmin};
    __syncthreads();
    SelPart r = s_w[0];
    for (int x = 1; x < kSelWaves; ++x) sel_merge(r.f, r.p, r.i, s_w[x].f, s_w[x].p, s_w[x].i);
    const double Fmin = r.f;
    const int32_t Pmin = r.p;
    const uint32_t iPmin = r.i;
    const double thr = Fmin * (1.0 + kTau);

    // the first band member lies in the first combine block (they cover
    // contiguous runs of scan indices in order) whose minimum is in the band
    uint32_t bfirst = my_f <= thr ? (uint32_t)threadIdx.x : UINT_MAX;
    for (int o = 32; o > 0; o >>= 1) bfirst = min(bfirst, (uint32_t)__shfl_xor((int)bfirst, o));
    if (lane == 0) s_first[wave] = bfirst;
    __syncthreads();
    for (int x = 0; x < kSelWaves; ++x) bfirst = min(bfirst, s_first[x]);
    uint32_t lo, hi;
    comb_range(n, comb_blocks, comb_group, bfirst, lo, hi);
    __syncthreads();                    // s_first is reused below

    // first scan index inside the band within [lo, hi): rounds of
    // 8 * NT indices, each thread's eight loads issued together;
    // the first round with a hit holds the answer
    uint32_t ifirst = UINT_MAX;
    for (uint32_t i0 = lo; i0 < hi; i0 += 8 * NT) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t i = i0 + u * NT + threadIdx.x;
            v[u] = i < hi ? be.F[i] : INFINITY;
        }
#pragma unroll
        for (int u = 7; u >= 0; --u)
            if (v[u] <= thr) ifirst = i0 + u * NT + threadIdx.x;
        if (__syncthreads_or(ifirst != UINT_MAX)) break;
    }
    for (int o = 32; o > 0; o >>= 1) ifirst = min(ifirst, (uint32_t)__shfl_xor((int)ifirst, o));
    if (lane == 0) s_first[wave] = ifirst;
    __syncthreads();
    uint32_t ib = s_first[0];
    for (int x = 1; x < kSelWaves; ++x) ib = min(ib, s_first[x]);
    // with finite F the block holding F_min is in the band, so a member was
    // found; the clamp only keeps the reads below in bounds otherwise
    ib = ib < n ? ib : iPmin < n ? iPmin : 0u;
    const uint32_t kb = (uint32_t)(((uint64_t)start + 1u + ib) % L);
    const uint32_t jp = (uint32_t)(((uint64_t)start + 1u + iPmin) % L);

    __shared__ int s_improve;
    if (threadIdx.x == 0) {
        be.near[0] = 0;           // the evaluation has read it; k_chunks appends to it
        const double Fb = be.F[ib];
        const int32_t Pb = be.P[ib];
        if (pure) {
            ChoiceDev c;
            c.i_best = ib; c.j_best = kb; c.F_best = Fb; c.F_min = Fmin;
            c.j_psl = jp; c.psl_min = Pmin; c.psl_k = Pb; c.flags = 0;
            out[bi] = c;
            s_improve = 0;
        } else {
            w.start = start;
            w.k = kb;
            w.i_best = ib;
            w.value_step = Fb;
            w.F_min = Fmin;
            w.psl_k = Pb;
            w.j_psl = jp;
            w.psl_min = Pmin;
            // three-way comparison of the move with v_local (Algorithm 1)
            uint32_t fl = 0;
            if (Fb < w.value_local * (1.0 - kTau)) fl = STEP_IMPROVED;
            else if (Fb > w.value_local * (1.0 + kTau)) fl = STEP_WORSE;
            w.flags = fl;
            s_improve = Pmin < w.psl_best;
            if (s_improve) {
                w.psl_best = Pmin;
                w.flags |= STEP_PSL_IMPROVED;
            }
        }
    }
    __syncthreads();
    if (s_improve) copy_words(w.best, w.pivot, w.nw, threadIdx.x, NT, jp >> 6, 1ull << (jp & 63u));
}

// ------------------------------------------------------- ambiguity flags

// The ambiguity flags of a step's scan, from the selection's results (by the
// block that made the selection, after it and before the flip and the
// bookkeeping):
//   ARGMIN: some scanned neighbour's F lies within amb = margin*F_min of the
//     band edge thr = F_min*(1+tau) (|F - thr| <= amb): a different rounding
//     of Eq. (5) could move it across the edge and change the move;
//   COMPARE (steps only): the move's F lies strictly within margin*v_local of
//     v_local*(1-tau) or of v_local*(1+tau), the edges of the three-way
//     comparison with the local best.
// Every F of a combine block is at least that block's minimum, so only the
// blocks whose minimum is at most thr + amb are read. pure != 0: the flag
// goes into the choice record out[b]; otherwise into the walk's step flags.
// Made by a block of NT threads.
template <int NT>
__device__ __forceinline__ void ambig_walk(WalkDev &w, const BatchEntry &be, uint32_t bi, uint32_t comb_blocks,
                                           uint32_t comb_group, int pure, ChoiceDev *out, double margin)
{
    const uint32_t n = be.fixed ? be.n_lmt : w.n_lmt;
    const double Fmin = pure ? out[bi].F_min : w.F_min;
    const double thr = Fmin * (1.0 + kTau), amb = margin * Fmin;
    // the combine blocks whose minimum lies at or below thr + amb, one per
    // thread (comb_blocks <= NT), as one 64-bit mask per wavefront
    static_assert(kCombMaxBlocks <= NT, "one combine block per thread");
    __shared__ uint64_t s_near[NT / 64];
    const uint32_t t = threadIdx.x;
    const bool near = t < comb_blocks && be.red[t].f - thr <= amb;
    const uint64_t m = __ballot(near);
    if ((t & 63) == 0) s_near[t >> 6] = m;
    __syncthreads();
    int hit = 0;
    for (uint32_t q = 0; q < NT / 64; ++q) {
        for (uint64_t bits = s_near[q]; bits; bits &= bits - 1) {   // the same for every thread of the block
            const uint32_t b = 64 * q + (uint32_t)__builtin_ctzll(bits);
            uint32_t lo, hi;
            comb_range(n, comb_blocks, comb_group, b, lo, hi);
            for (uint32_t i = lo + t; i < hi; i += NT) {
                const double g = be.F[i] - thr;
                hit |= (g < 0.0 ? -g : g) <= amb;
            }
        }
    }
    hit = __syncthreads_or(hit);
    if (threadIdx.x == 0) {
        if (pure) {
            out[bi].flags = hit ? CHOICE_AMBIG_ARGMIN : 0u;
        } else {
            uint32_t fl = w.flags;
            if (hit) fl |= STEP_AMBIG_ARGMIN;
            const double vl = w.value_local, v = w.value_step;
            const double elo = vl * (1.0 - kTau), ehi = vl * (1.0 + kTau), band = margin * vl;
            if ((v - elo < band && elo - v < band) || (v - ehi < band && ehi - v < band)) fl |= STEP_AMBIG_COMPARE;
            w.flags = fl;
        }
    }
}

// The rest of one loop iteration of Algorithm 1 after the selection, by the
// block of NT threads that made it (batch position bi): the move's bit, the
// three-way comparison with v_local, the unimproved counter, the local best,
// and the phase switch (Rand_flip of the local best and the exponent swap;
// the walk joins the batch's pending list, whose C, F and PSL k_pending then
// rebuilds). The C update runs after it (k_apply), from bits that equal the
// pre-move pivot's at every position but j: the pivot's, or on a switch the
// local best's (which are then the move's pivot, if the move improved; if it
// did not, C is rebuilt from C of the local best anyway).
template <int NT>
__device__ __forceinline__ void bookkeep_walk(WalkDev &w, uint32_t bi, uint32_t *pend)
{
    __shared__ int s_improved, s_switch;
    __shared__ uint32_t s_pos[1024];
    if (threadIdx.x == 0) {
        const uint32_t k = w.k;
        w.pivot[k >> 6] ^= 1ull << (k & 63u);
        w.F_pivot = w.value_step;
        w.psl_pivot = w.psl_k;
        // the comparison with v_local was taken by the selection
        int improved = 0, sw = 0;
        uint32_t flags = w.flags;
        if (flags & STEP_IMPROVED) {
            improved = 1;
            w.unimproved = 0;
            w.value_local = w.value_step;
        } else if (flags & STEP_WORSE) {
            w.unimproved += 1;
            if (w.switch_period == 0 && w.unimproved > w.ls_lmt) sw = 1;
        }
        if (w.switch_period > 0 && ((w.t + 1u) % w.switch_period) == 0) sw = 1;
        if (sw) flags |= STEP_SWITCHED;
        w.flags = flags;
        if (w.trace_cap) {
            TraceEntry e;
            e.t = w.t;
            e.start = w.start;
            e.k = w.k;
            e.value_step = w.value_step;
            e.psl_k = w.psl_k;
            e.psl_best = w.psl_best;
            e.alpha = sw ? (w.alpha == w.alpha1 ? w.alpha2 : w.alpha1) : w.alpha;
            e.flags = flags;
            w.trace[w.t % w.trace_cap] = e;
        }
        w.t += 1;
        s_improved = improved;
        s_switch = sw;
    }
    __syncthreads();
    if (s_improved) copy_words(w.local_best, w.pivot, w.nw, threadIdx.x, NT, UINT32_MAX, 0);
    __syncthreads();
    if (s_switch) {
        copy_words(w.pivot, w.local_best, w.nw, threadIdx.x, NT, UINT32_MAX, 0);
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t L = w.L;
            uint32_t cnt = 0;
            for (uint64_t r = 0; cnt < w.flip_lmt && r < (1ull << 24); ++r) {
                const uint64_t ctr = (2ull << 60) | (w.q << 24) | r;
                const uint32_t pos = (uint32_t)(draw(w.seed, ctr) % (uint64_t)L);
                bool dup = false;
                for (uint32_t x = 0; x < cnt; ++x) dup |= (s_pos[x] == pos);
                if (dup) continue;
                s_pos[cnt] = pos;
                w.flips[cnt] = pos;
                ++cnt;
                w.pivot[pos >> 6] ^= 1ull << (pos & 63u);
            }
            w.n_flips = cnt;
            w.alpha = (w.alpha == w.alpha1) ? w.alpha2 : w.alpha1;
            w.q += 1;
            w.pending = 1;
            pend[1 + atomicAdd(&pend[0], 1u)] = bi;
        }
    }
}

// F and PSL per candidate from the k-split partials, spread over gridDim.x
// blocks per walk (blockIdx.y = batch position); each block leaves its
// smallest F and its first smallest PSL in be.red. A group of G lanes
// (a power of two, at most 64) shares a candidate: lane g adds splits g,
// g+G, ... in order, then the group adds its lanes' sums in a fixed order for
// a given split count and G (G = 1 adds the splits in order). For G <= 4 a
// group is G adjacent lanes (a butterfly); for G >= 8 a block pass takes
// cpb = 256 / G <= 32 candidates, lane t of the block has candidate t mod cpb
// and split lane t / cpb, so that one load of a wavefront reads cpb
// consecutive partials of each of 64 / cpb splits; the sums go through a
// butterfly over the wavefront's split lanes, then the four wavefronts' sums
// are added in wavefront order.
// With tail != 0 the walk's last block to finish then makes its selection
// (select_walk) and its ambiguity flags; b0 = the batch position of
// blockIdx.y = 0; done holds one zeroed counter per batch position.
__global__ __launch_bounds__(kCombThreads) void k_combine(WalkDev *walks, const BatchEntry *batch, Tables tabs,
                                                          int G, int tail, int pure, ChoiceDev *out, uint32_t *pend,
                                                          uint32_t *done, double margin, uint32_t b0)
{
    const BatchEntry be = batch[blockIdx.y];
    WalkDev &w = walks[be.slot];
    const uint32_t n = be.fixed ? be.n_lmt : w.n_lmt;
    const uint32_t ks = be.ksplit;
    const double *T = tabs.T[w.alpha];
    const uint32_t cpb = kCombThreads / (uint32_t)G;      // candidates per block pass
    const bool wide = G >= 8;
    const uint32_t g = wide ? threadIdx.x / cpb : threadIdx.x & (uint32_t)(G - 1);
    const uint32_t ci = wide ? threadIdx.x % cpb : threadIdx.x / (uint32_t)G;   // candidate in the pass
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    static_assert(kCombThreads == 256, "four wavefronts per combine block");
    __shared__ double s_wf[4][32];
    __shared__ uint32_t s_wm[4][32];
    // split path: the partials hold the VALU terms only; the prefix sums and
    // the linear sums (psl_split.hip) supply the rest of F_j
    const bool split = be.lsplit != 0 && be.ss->use != 0;
    const double U = split ? be.ss->U : 0.0;
    const uint32_t start = be.fixed ? be.start : step_start(w);
    const uint32_t L = w.L;

    double fmin = INFINITY;
    int32_t pmin = INT_MAX;
    uint32_t ipmin = UINT_MAX;
    uint32_t lo, hi;
    comb_range(n, gridDim.x, (uint32_t)G, blockIdx.x, lo, hi);
    for (uint32_t i0 = lo; i0 < hi; i0 += cpb) {
        const uint32_t i = i0 + ci;
        double f = 0.0;
        uint32_t m = 0;
        if (i < hi) {
            // up to kCombBatch of this lane's splits are loaded before they
            // are added (in split order)
            for (uint32_t x0 = g; x0 < ks; x0 += (uint32_t)G * kCombBatch) {
                double v[kCombBatch];
                uint32_t mv[kCombBatch];
#pragma unroll
                for (int u = 0; u < kCombBatch; ++u) {
                    const uint32_t x = x0 + (uint32_t)u * (uint32_t)G;
                    if (x < ks) {
                        v[u] = be.Fpart[(size_t)x * n + i];
                        mv[u] = be.Mpart[(size_t)x * n + i];
                    }
                }
#pragma unroll
                for (int u = 0; u < kCombBatch; ++u) {
                    if (x0 + (uint32_t)u * (uint32_t)G < ks) {
                        f += v[u];
                        m = max(m, mv[u]);
                    }
                }
            }
        }
        if (wide) {
            for (int o = (int)cpb; o < 64; o <<= 1) {
                f += __shfl_xor(f, o);
                m = max(m, (uint32_t)__shfl_xor((int)m, o));
            }
            if ((uint32_t)lane < cpb) {
                s_wf[wave][lane] = f;
                s_wm[wave][lane] = m;
            }
            __syncthreads();
            if (g == 0) {           // wavefront 0, lanes below cpb
                f = s_wf[0][lane];
                m = s_wm[0][lane];
                for (int x = 1; x < 4; ++x) {
                    f += s_wf[x][lane];
                    m = max(m, s_wm[x][lane]);
                }
            }
            __syncthreads();        // the next pass rewrites the rows
        } else {
            for (int o = G >> 1; o > 0; o >>= 1) {
                f += __shfl_xor(f, o);
                m = max(m, (uint32_t)__shfl_xor((int)m, o));
            }
        }
        if (g == 0 && i < hi) {
            // the near-peak path stores the PSL itself; the dense path the
            // high word of T(PSL), which is at least hi32(T(1)) = 0x3FF00000
            // because |C'_{L-1}| = 1 for every sequence
            const int32_t p = m < 0x3FF00000u ? (int32_t)m : table_inverse(T, tabs.n, m);
            if (split) {
                // F_j = sum_{k<=m} A_k + sum_{m<k<=M} A'_k + sum_{k>M} T(|C_k|)
                //       - s_j U (linear sums) + the VALU terms, m = min(j, L-1-j)
                const uint32_t j = (uint32_t)(((uint64_t)start + 1u + i) % L);
                const uint32_t mj = min(j, L - 1 - j), Mj = max(j, L - 1 - j);
                const double *pa = be.pre, *pa1 = be.pre + L, *pt = be.pre + 2 * (size_t)L;
                const double cst = pa[mj] + (pa1[Mj] - pa1[mj]) + (pt[L - 1] - pt[Mj]);
                double lin = 0.0;
                for (uint32_t x = 0; x < be.lsplit; ++x) lin += be.lpart[(size_t)x * L + j];
                const double sgn = get_bit(w.pivot, j) ? U : -U;     // -s_j U
                f = cst + sgn * lin + f;
            }
            be.F[i] = f;
            be.P[i] = p;
            fmin = f < fmin ? f : fmin;
            if (p < pmin) { pmin = p; ipmin = i; }
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double of = __shfl_xor(fmin, o);
        const int32_t op = __shfl_xor(pmin, o);
        const uint32_t oi = (uint32_t)__shfl_xor((int)ipmin, o);
        sel_merge(fmin, pmin, ipmin, of, op, oi);
    }
    __shared__ SelPart s_r[kCombThreads / 64];
    if (lane == 0) s_r[wave] = SelPart{fmin, pmin, ipmin};
    __syncthreads();
    if (threadIdx.x == 0) {
        SelPart r = s_r[0];
        for (int x = 1; x < kCombThreads / 64; ++x) sel_merge(r.f, r.p, r.i, s_r[x].f, s_r[x].p, s_r[x].i);
        be.red[blockIdx.x] = r;
    }
    if (!tail) return;
    // tail != 0: the walk's last block to finish (counted in done[bi], which
    // it returns to 0 for the next launch) makes the selection and sets the
    // ambiguity flags. Each block's count is a device-scope release of its F,
    // P and minimum, and the last block acquires them all.
    const uint32_t bi = b0 + blockIdx.y;
    __shared__ uint32_t s_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t last = 1;
        if (gridDim.x > 1) {
            const uint32_t before =
                __hip_atomic_fetch_add(&done[bi], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            last = before == gridDim.x - 1 ? 1u : 0u;
            if (last) done[bi] = 0;
        }
        s_last = last;
    }
    __syncthreads();
    if (!s_last) return;
    if (gridDim.x > 1) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    select_walk<kCombThreads>(w, be, bi, gridDim.x, (uint32_t)G, pure, out);
    __syncthreads();
    ambig_walk<kCombThreads>(w, be, bi, gridDim.x, (uint32_t)G, pure, out, margin);
    if (!pure) {
        __syncthreads();
        bookkeep_walk<kCombThreads>(w, bi, pend);
    }
}

// The selection of a walk, its ambiguity flags and (pure == 0) its
// bookkeeping: one block per walk, after k_combine when the combine launch
// does not make them itself.
constexpr int kSelThreads = 256;
__global__ __launch_bounds__(kSelThreads) void k_select(WalkDev *walks, const BatchEntry *batch,
                                                        uint32_t comb_blocks, uint32_t comb_group, int pure,
                                                        ChoiceDev *out, uint32_t *pend, double margin)
{
    const BatchEntry be = batch[blockIdx.x];
    WalkDev &w = walks[be.slot];
    select_walk<kSelThreads>(w, be, blockIdx.x, comb_blocks, comb_group, pure, out);
    __syncthreads();
    ambig_walk<kSelThreads>(w, be, blockIdx.x, comb_blocks, comb_group, pure, out, margin);
    if (!pure) {
        __syncthreads();
        bookkeep_walk<kSelThreads>(w, blockIdx.x, pend);
    }
}


// ------------------------------------------------------------ flip

// Flip(pivot, j), part 1: C_k += -2 s_j (s_{j+k} + s_{j-k}) over the terms in
// bounds, read from the pivot before its bit changes. j_fixed < 0: the walk's
// recorded move.
constexpr int kApplyThreads = 256;

// The C update of shifts k0 + tid, k0 + tid + kApplyThreads, ... < k1. C and
// C_lb are separate arrays: each thread loads four shifts' C values and bit
// words before it stores any of them. The bit words of j + k and j - k are
// read whether or not those elements exist: the pivot's zero guard words
// (nw + 2 on each side) hold every index from -(L-1) to 2L-2.
constexpr int kApplyBatch = 4;
__device__ __forceinline__ void apply_range(int32_t *__restrict__ C, int32_t *__restrict__ C_lb,
                                            const uint64_t *__restrict__ b, uint32_t L, uint32_t j, int sj,
                                            bool lb, uint32_t k0, uint32_t k1)
{
    for (uint32_t k = k0 + threadIdx.x; k < k1; k += kApplyBatch * kApplyThreads) {
        int32_t cv[kApplyBatch];
        uint64_t wr[kApplyBatch], wl[kApplyBatch];
#pragma unroll
        for (int u = 0; u < kApplyBatch; ++u) {
            uint32_t kk = k + (uint32_t)u * kApplyThreads;
            kk = kk < k1 ? kk : k;                  // past the end: a valid shift, not stored
            const int32_t pl = (int32_t)j - (int32_t)kk;
            cv[u] = C[kk];
            wr[u] = b[(j + kk) >> 6];
            wl[u] = b[pl >> 6];                     // arithmetic shift: a guard word when pl < 0
        }
#pragma unroll
        for (int u = 0; u < kApplyBatch; ++u) {
            const uint32_t kk = k + (uint32_t)u * kApplyThreads;
            if (kk < k1) {
                int d = 0;
                if (j + kk < L) d += ((wr[u] >> ((j + kk) & 63u)) & 1u) ? -1 : 1;
                if (kk <= j) d += ((wl[u] >> ((j - kk) & 63u)) & 1u) ? -1 : 1;
                const int32_t c = cv[u] - 2 * sj * d;
                C[kk] = c;
                if (lb) C_lb[kk] = c;
            }
        }
    }
}


__global__ __launch_bounds__(kApplyThreads) void k_apply(WalkDev *walks, const BatchEntry *batch,
                                                         int64_t j_fixed, SegMap map)
{
    uint32_t bi, seg;
    seg_of(map, blockIdx.x, bi, seg);
    WalkDev &w = walks[batch[bi].slot];
    const uint32_t L = w.L;
    const uint32_t j = j_fixed >= 0 ? (uint32_t)j_fixed : w.k;
    // a forced flip reads the pivot before its bit changes; the step's move
    // comes after the bookkeeping, which flipped bit j, and on a phase switch
    // replaced the pivot: then the local best holds the pre-move bits at
    // every position but j (an improving move), or C is rebuilt afterwards
    const bool moved = j_fixed < 0;
    const uint64_t *b = moved && (w.flags & STEP_SWITCHED) ? w.local_best : w.pivot;
    const int sj = (get_bit(b, j) != 0) != moved ? -1 : 1;      // s_j before the flip
    // the move improves on v_local: the new pivot becomes local_best
    const bool lb = moved && (w.flags & STEP_IMPROVED);
    const uint32_t k0 = 1u + (seg << map.shift);
    const uint32_t k1 = min(L, k0 + (1u << map.shift));
    apply_range(w.C, w.C_lb, b, L, j, sj, lb, k0, k1);
}

// Flip(pivot, j), part 2, for a forced flip: the bit itself.
__global__ void k_flip_bit(WalkDev *walks, const BatchEntry *batch, uint32_t j)
{
    WalkDev &w = walks[batch[0].slot];
    if (threadIdx.x == 0) w.pivot[j >> 6] ^= 1ull << (j & 63u);
}

// ------------------------------------------------------------ launches

hipError_t launch_power_table(double *T, uint32_t n, uint32_t alpha, hipStream_t s)
{
    k_power_table<<<(n + 255) / 256, 256, 0, s>>>(T, n, alpha);
    return hipGetLastError();
}

hipError_t launch_init_bits(WalkDev *walks, const BatchEntry *batch, const uint32_t *want,
                            uint32_t nb, uint32_t max_nw, hipStream_t s)
{
    for (uint32_t b0 = 0; b0 < nb; b0 += kMaxGridY) {
        k_init_bits<<<dim3((max_nw + 255) / 256, std::min(kMaxGridY, nb - b0)), 256, 0, s>>>(walks, batch + b0,
                                                                                             want + b0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_corr(WalkDev *walks, const BatchEntry *batch, uint32_t nb, uint32_t max_L,
                       int only_pending, hipStream_t s)
{
    for (uint32_t b0 = 0; b0 < nb; b0 += kMaxGridY) {
        k_corr<<<dim3((max_L + kCorrThreads - 1) / kCorrThreads, std::min(kMaxGridY, nb - b0)), kCorrThreads, 0,
                 s>>>(walks, batch + b0, only_pending);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_pending(WalkDev *walks, const BatchEntry *batch, uint32_t nb, uint64_t units,
                          const Tables &tabs, const uint32_t *pend, hipStream_t s)
{
    if (!pend) return hipErrorInvalidValue;
    // every unit of the batch's walks gets a block when all of them switch
    const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(4096, units));
    k_pending<<<grid, kPendThreads, 0, s>>>(walks, batch, tabs, pend);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_pending_fin<<<std::max<uint32_t>(1, std::min<uint32_t>(nb, 1024)), 64, 0, s>>>(walks, batch, pend);
    return hipGetLastError();
}

hipError_t launch_fitness(WalkDev *walks, const BatchEntry *batch, uint32_t nb, const Tables &tabs,
                          int mode, hipStream_t s)
{
    k_fitness<<<nb, kFitThreads, 0, s>>>(walks, batch, tabs, mode);
    return hipGetLastError();
}

hipError_t launch_suffix(WalkDev *walks, const BatchEntry *batch, uint32_t nb, uint32_t max_L,
                         const Tables &tabs, int mode, const SegMap *map, uint32_t *pend, int scan, hipStream_t s)
{
    if (mode != 0 && mode != 2) return hipErrorInvalidValue;
    if (!map || map->total == 0 || map->nb != nb || map->shift < kSegShiftMin || map->shift > kSegShiftMax)
        return hipErrorInvalidValue;
    scan = mode == 0 && scan;
    if (scan && (!map->tot || !map->tmax)) return hipErrorInvalidValue;
    SegMap m = *map;
    if (!scan) m.tot = nullptr, m.tmax = nullptr;
    k_chunks<<<m.total, kChunkThreads, 0, s>>>(walks, batch, tabs, mode, m, mode == 0 ? pend : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (scan) {
        // suffix values segment by segment (evaluations in 16-wavefront blocks)
        constexpr uint32_t per = kSegScanThreads / 64;
        k_seg_scan<<<(m.total + per - 1) / per, kSegScanThreads, 0, s>>>(walks, batch, m);
    } else if (mode == 2) {
        // the initial fitness: totals per walk
        k_scan<<<nb, kScanThreads, 0, s>>>(walks, batch);
    }
    return hipGetLastError();
}

__global__ void k_near_reset(const BatchEntry *batch, uint32_t nb, uint32_t *pend, uint32_t *done)
{
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) batch[b].near[0] = 0;
    if (b < nb && done) done[b] = 0;
    if (b == 0 && pend) pend[0] = 0;
}

hipError_t launch_near_reset(const BatchEntry *batch, uint32_t nb, uint32_t *pend, uint32_t *done, hipStream_t s)
{
    k_near_reset<<<(nb + 255) / 256, 256, 0, s>>>(batch, nb, pend, done);
    return hipGetLastError();
}

hipError_t launch_select(WalkDev *walks, const BatchEntry *batch, uint32_t nb, uint32_t comb_blocks,
                         uint32_t comb_group, const Tables &tabs, int pure, void *out, uint32_t *pend,
                         uint32_t *done, double margin, hipStream_t s)
{
    if (comb_blocks < 1 || comb_blocks > kCombMaxBlocks) return hipErrorInvalidValue;
    if (comb_group < 1 || comb_group > 64 || (comb_group & (comb_group - 1))) return hipErrorInvalidValue;
    if (pure && (!out || nb != 1)) return hipErrorInvalidValue;
    if (nb == 0) return hipSuccess;
    // small launches make the selection in the combine launch (one launch
    // fewer); large ones in launches of their own, where the per-block
    // device-scope release of the fused form costs more than the launches
    const int tail = comb_blocks == 1 || ((uint64_t)nb * comb_blocks <= kCombFuseBlocks && done) ? 1 : 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += kMaxGridY) {
        k_combine<<<dim3(comb_blocks, std::min(kMaxGridY, nb - b0)), kCombThreads, 0, s>>>(
            walks, batch + b0, tabs, (int)comb_group, tail, pure, (ChoiceDev *)out, pend, done, margin, b0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (tail) return hipSuccess;
    k_select<<<nb, kSelThreads, 0, s>>>(walks, batch, comb_blocks, comb_group, pure, (ChoiceDev *)out, pend,
                                        margin);
    return hipGetLastError();
}

size_t choice_dev_size() { return sizeof(ChoiceDev); }

void choice_dev_unpack(const void *p, uint32_t *i_best, uint32_t *j_best, double *F_best,
                       double *F_min, uint32_t *j_psl, int32_t *psl_min, int32_t *psl_k, uint32_t *flags)
{
    const ChoiceDev *c = (const ChoiceDev *)p;
    *i_best = c->i_best; *j_best = c->j_best; *F_best = c->F_best; *F_min = c->F_min;
    *j_psl = c->j_psl; *psl_min = c->psl_min; *psl_k = c->psl_k; *flags = c->flags;
}

hipError_t launch_apply(WalkDev *walks, const BatchEntry *batch, const SegMap &map, int64_t j_fixed,
                        hipStream_t s)
{
    if (map.shift < kSegShiftMin || map.shift > kSegShiftMax) return hipErrorInvalidValue;
    if (map.total == 0) return hipSuccess;       // L = 1 has no shift to update
    k_apply<<<map.total, kApplyThreads, 0, s>>>(walks, batch, j_fixed, map);
    return hipGetLastError();
}

hipError_t launch_flip_bit(WalkDev *walks, const BatchEntry *batch, uint32_t j, hipStream_t s)
{
    k_flip_bit<<<1, 64, 0, s>>>(walks, batch, j);
    return hipGetLastError();
}


}  // namespace psl
