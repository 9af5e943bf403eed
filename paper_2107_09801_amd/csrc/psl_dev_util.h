// psl_dev_util.h -- small device helpers shared by the libpsl kernel sources
// (internal).
#pragma once

#include "psl_device.h"

namespace psl {

// Counter-based SplitMix64 (Steele, Lea & Flood 2014): output ctr+1 of the
// stream whose state starts at seed.
__device__ __forceinline__ uint64_t draw(uint64_t seed, uint64_t ctr)
{
    uint64_t z = seed + (ctr + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t step_start(const WalkDev &w)
{
    return (uint32_t)(draw(w.seed, (1ull << 60) | w.t) % (uint64_t)w.L);
}

__device__ __forceinline__ uint32_t get_bit(const uint64_t *b, uint32_t i)
{
    return (uint32_t)((b[i >> 6] >> (i & 63u)) & 1u);
}

// dst[x] = src[x] for x < n (word flip_word also XORed with flip_mask), the
// threads of a block striding by nthreads. The two arrays never overlap;
// each thread issues eight loads before their stores instead of waiting on
// one load per word.
__device__ __forceinline__ void copy_words(uint64_t *__restrict__ dst, const uint64_t *__restrict__ src,
                                           uint32_t n, uint32_t tid, uint32_t nthreads, uint32_t flip_word,
                                           uint64_t flip_mask)
{
    uint32_t x = tid;
    for (; x + 7u * nthreads < n; x += 8u * nthreads) {
        uint64_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = src[x + (uint32_t)u * nthreads];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t y = x + (uint32_t)u * nthreads;
            dst[y] = y == flip_word ? v[u] ^ flip_mask : v[u];
        }
    }
    for (; x < n; x += nthreads) dst[x] = x == flip_word ? src[x] ^ flip_mask : src[x];
}

// Bits [pos, pos+32) of a packed sequence held as nw32 32-bit words; bits
// outside the words read as 0.
__device__ __forceinline__ uint32_t bits32_at(const uint32_t *__restrict__ w32, int nw32,
                                              int pos)
{
    int wi = pos >> 5;
    uint32_t sh = (uint32_t)pos & 31u;
    uint32_t lo = (wi >= 0 && wi < nw32) ? w32[wi] : 0u;
    uint32_t hi = (wi + 1 >= 0 && wi + 1 < nw32) ? w32[wi + 1] : 0u;
    return __builtin_amdgcn_alignbit(hi, lo, sh);
}

__device__ __forceinline__ double dmax(double a, double b) { return a > b ? a : b; }

// High 32 bits of a non-negative double. Over the power table they are
// strictly increasing in |c| (consecutive entries differ by a factor of at
// least 1 + 2^-19 for alpha >= 2 and |c| <= 2^20 + 8; for alpha = 1 the
// entries are integers below 2^21, exact in 20 fraction bits), so the
// running maximum of T(|C'|) can be kept as a 32-bit unsigned maximum.
__device__ __forceinline__ uint32_t hi32(double v)
{
    return (uint32_t)((uint64_t)__double_as_longlong(v) >> 32);
}

// Neumaier's compensated addition.
__device__ __forceinline__ void nsum_add(double &sum, double &comp, double x)
{
    double t = sum + x;
    if (fabs(sum) >= fabs(x)) comp += (sum - t) + x;
    else                      comp += (x - t) + sum;
    sum = t;
}

// Smallest c with hi32(T[c]) >= h: |c| from the high word of T(|c|).
__device__ __forceinline__ int32_t table_inverse(const double *T, uint32_t n, uint32_t h)
{
    uint32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (hi32(T[mid]) < h) lo = mid + 1;
        else                  hi = mid;
    }
    return (int32_t)lo;
}

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of work items so that the blocks of one walk share an L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nb)
{
    const uint32_t nx = 8;
    uint32_t q = nb / nx, r = nb % nx;
    uint32_t x = b % nx, local = b / nx;
    return x * q + (x < r ? x : r) + local;
}

// (walk, segment) of block i of an O(L) pass.
__device__ __forceinline__ void seg_of(const SegMap &m, uint32_t i, uint32_t &b, uint32_t &seg)
{
    if (!m.off) {
        b = i / m.spw;
        seg = i - b * m.spw;
        return;
    }
    uint32_t lo = 0, hi = m.nb - 1;      // the largest b with off[b] <= i
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (m.off[mid] <= i) lo = mid;
        else                 hi = mid - 1;
    }
    b = lo;
    seg = i - m.off[lo];
}


// The last both-neighbour shift of the aligned 64-element block holding j:
// min over j' of the block of min(j', L-1-j') (a tent function, so the
// minimum over an interval is at one of its ends). A 32-shift chunk
// 1+32c .. 32+32c is "covered" for the block when it ends at or below this
// bound; the linear items then use B_k for it instead of B'_k (psl_split.hip
// makes the same choice per block and chunk).
__device__ __forceinline__ int split_block_bound(int j, int L)
{
    const int j0 = j & ~63, j1 = min(j0 + 63, L - 1);
    return min(min(j0, L - 1 - j0), min(j1, L - 1 - j1));
}

}  // namespace psl
