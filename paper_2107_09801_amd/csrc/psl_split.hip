// psl_split.hip -- the split evaluation of libpsl (gfx950).
//
// Eq. (5) summed over the neighbours of Algorithm 1, regrouped. For shift k
// with c = C_k and T(x) = T_alpha(|x|), the one-element flip of Section 3
// changes C_k by 2a + 2b when both neighbours of j exist and by 2a when one
// does (a, b = +-1: a = -s_j s_{j+k}, b = -s_j s_{j-k}). Because a and b
// are +-1, each term is exactly a polynomial in them:
//   T(|c + 2a + 2b|) = A + B (a + b) + D ab,
//     A = (T(c+4) + 2T(c) + T(c-4))/4, B = (T(c+4) - T(c-4))/4,
//     D = (T(c+4) + T(c-4) - 2T(c))/4;
//   T(|c + 2a|) = A' + B' a, A' = (T(c+2) + T(c-2))/2, B' = (T(c+2) - T(c-2))/2.
// So F_j = (prefix sums of A, A', T at j's region bounds)
//        - s_j (sum_k beta_k s_{j+k} + sum_k beta_k s_{j-k})   [the linear part]
//        + sum over both-neighbour shifts of D_k ab (+ (B_k - B'_k)(a + b)
//          where the linear part used B'_k).
// The linear part is a sum of products of +-1 elements and coefficients:
// the matrix cores take it as exact integers (B and B' quantized to
// multiples of a power of two U, kLimbs signed byte digits each). This file
// holds the per-step preparation (coefficients, digits, prefix sums, scale
// and path choice) and the matrix-core kernel of the linear part.
#include "psl_dev_util.h"
#include "psl_device.h"
#include "psl_launch.h"

#include <algorithm>
#include <climits>

namespace psl {

// The scale of step's quantized coefficients: U = 2^e with every |B_k| and
// |B'_k| below 2^62 U. Both grow with |c| (T is increasing and convex in
// |c|), so their largest values are those at |c| = P, the pivot's PSL (the
// maximum |C_k|).
__device__ __forceinline__ double split_scale(const double *__restrict__ T, int P)
{
    const int m4 = P >= 4 ? P - 4 : 4 - P, m2 = P >= 2 ? P - 2 : 2 - P;
    const double b1 = (T[P + 4] - T[m4]) * 0.25, b2 = (T[P + 2] - T[m2]) * 0.5;
    const double bmax = b1 > b2 ? b1 : b2;
    return ldexp(1.0, ilogb(bmax) - 61);
}

// The kLimbs balanced base-256 digits (each in [-128, 127]) of q.
__device__ __forceinline__ void split_digits(int64_t q, int8_t *__restrict__ out, size_t stride)
{
#pragma unroll
    for (int l = 0; l < kLimbs; ++l) {
        const int d = (int)((q + 128) & 0xFF) - 128;
        out[(size_t)l * stride] = (int8_t)d;
        q = (q - d) >> 8;
    }
}

// Per shift k of every split walk of the batch (one block per segment of a
// walk's shifts): the digits of B'_k and B_k, D_k and B_k - B'_k, and the
// values A_k, A'_k, T(|C_k|) that k_split_scan turns into prefix sums.
constexpr int kPrepThreads = 256;
__global__ __launch_bounds__(kPrepThreads) void k_split_prep(const WalkDev *walks, const BatchEntry *batch,
                                                             Tables tabs, SegMap map)
{
    uint32_t b, seg;
    seg_of(map, blockIdx.x, b, seg);
    const BatchEntry be = batch[b];
    if (!be.lsplit) return;
    const WalkDev &w = walks[be.slot];
    const int L = (int)w.L;
    const double *__restrict__ T = tabs.T[w.alpha];
    const double U = split_scale(T, w.psl_pivot);
    const double inv = 1.0 / U;                    // exact: U is a power of two
    const size_t K = split_row((uint32_t)L);       // digits per (set, limb)
    const int k0 = 1 + (int)(seg << map.shift);
    const int k1 = min(L, k0 + (1 << map.shift));
    for (int k = k0 + (int)threadIdx.x; k < k1; k += kPrepThreads) {
        const int c = w.C[k];
        const int a4 = c + 4 < 0 ? -(c + 4) : c + 4, m4 = c - 4 < 0 ? 4 - c : c - 4;
        const int a2 = c + 2 < 0 ? -(c + 2) : c + 2, m2 = c - 2 < 0 ? 2 - c : c - 2;
        const int a0 = c < 0 ? -c : c;
        const double tp4 = T[a4], tm4 = T[m4], tp2 = T[a2], tm2 = T[m2], t0 = T[a0];
        const double A = (tp4 + 2.0 * t0 + tm4) * 0.25;
        const double B = (tp4 - tm4) * 0.25;
        const double D = (tp4 + tm4 - 2.0 * t0) * 0.25;
        const double A1 = (tp2 + tm2) * 0.5;
        const double B1 = (tp2 - tm2) * 0.5;
        split_digits(__double2ll_rn(B1 * inv), be.limbs + (k - 1), K);
        split_digits(__double2ll_rn(B * inv), be.limbs + (size_t)kLimbs * K + (k - 1), K);
        be.dq[2 * (size_t)k] = D;
        be.dq[2 * (size_t)k + 1] = B - B1;
        be.pre[k] = A;
        be.pre[(size_t)L + k] = A1;
        be.pre[2 * (size_t)L + k] = t0;
    }
    if (k1 == L) {
        // the shifts at and beyond L (the rest of the last chunk and the
        // zero chunk): zero digits
        for (int k = L + (int)threadIdx.x; k <= (int)K; k += kPrepThreads)
            for (int s = 0; s < 2 * kLimbs; ++s) be.limbs[(size_t)s * K + (k - 1)] = 0;
    }
}

// One block per (split walk, value array): the array becomes its inclusive
// prefix sums over k = 1..k (entry 0 = 0). Chunks of kScanChunk consecutive
// entries go through the block in order: each thread sums its kScanPer
// entries, the wavefronts scan their threads' totals and the block adds the
// wavefronts' totals before them, and the chunks' totals are carried with
// Neumaier's compensation. Every summand is non-negative, so each prefix is
// within a few dozen roundings of its exact value. Block (walk, 0) also
// stores the step's scale and path choice: the split path is taken when the
// near-peak list holds the PSL (sparse form) and the quantization error of
// the linear part, at most (L-1) U, is below 1e-14 of a lower bound of every
// neighbour's F (T(P-4) for the pivot's PSL P, and at least 1).
constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanChunk = kScanThreads * kScanPer;
__global__ __launch_bounds__(kScanThreads) void k_split_scan(const WalkDev *walks, const BatchEntry *batch,
                                                             Tables tabs)
{
    const uint32_t wb = blockIdx.x / 3, x = blockIdx.x % 3;
    const BatchEntry be = batch[wb];
    if (!be.lsplit) return;
    const WalkDev &w = walks[be.slot];
    const int L = (int)w.L;
    double *__restrict__ v = be.pre + (size_t)x * L;
    __shared__ double s_tot[kScanThreads / 64];
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    auto load = [&](int base, double (&e)[kScanPer]) {
        const int k0 = base + (int)threadIdx.x * kScanPer;
#pragma unroll
        for (int i = 0; i < kScanPer; ++i) e[i] = k0 + i < L ? v[k0 + i] : 0.0;
    };
    double carry = 0.0, ccomp = 0.0;
    double cur[kScanPer], nxt[kScanPer];
    load(1, cur);
    for (int base = 1; base < L; base += kScanChunk) {
        if (base + kScanChunk < L) load(base + kScanChunk, nxt);
#pragma unroll
        for (int i = 1; i < kScanPer; ++i) cur[i] += cur[i - 1];
        // inclusive scan of the thread totals over the wavefront
        double t = cur[kScanPer - 1];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double o = __shfl_up(t, d);
            if (lane >= d) t += o;
        }
        double excl = __shfl_up(t, 1);
        if (lane == 0) excl = 0.0;
        if (lane == 63) s_tot[wave] = t;
        __syncthreads();
        double off = carry + ccomp, tot = 0.0;
#pragma unroll
        for (int q = 0; q < kScanThreads / 64; ++q) {
            if (q < wave) off += s_tot[q];
            tot += s_tot[q];
        }
        off += excl;
        const int k0 = base + (int)threadIdx.x * kScanPer;
#pragma unroll
        for (int i = 0; i < kScanPer; ++i)
            if (k0 + i < L) v[k0 + i] = off + cur[i];
        nsum_add(carry, ccomp, tot);
        __syncthreads();                           // s_tot is rewritten by the next chunk
#pragma unroll
        for (int i = 0; i < kScanPer; ++i) cur[i] = nxt[i];
    }
    if (threadIdx.x == 0) {
        v[0] = 0.0;
        if (x == 0) {
            const double *__restrict__ T = tabs.T[w.alpha];
            const int P = w.psl_pivot;
            const double U = split_scale(T, P);
            const double flow = P > 4 ? T[P - 4] : 0.0;
            const bool exact_enough = (double)(L - 1) * U <= 1e-14 * (flow > 1.0 ? flow : 1.0);
            const bool sparse_psl = be.near[0] <= be.near_lim;
            SplitState st;
            st.U = U;
            st.use = exact_enough && sparse_psl ? 1u : 0u;
            st.pad = 0;
            *be.ss = st;
        }
    }
}

hipError_t launch_split_prep(const WalkDev *walks, const BatchEntry *batch, uint32_t nb, const Tables &tabs,
                             const SegMap &map, hipStream_t s)
{
    if (map.shift < kSegShiftMin || map.shift > kSegShiftMax || map.nb != nb) return hipErrorInvalidValue;
    if (nb == 0 || map.total == 0) return hipSuccess;
    k_split_prep<<<map.total, kPrepThreads, 0, s>>>(walks, batch, tabs, map);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_split_scan<<<3 * nb, kScanThreads, 0, s>>>(walks, batch, tabs);
    return hipGetLastError();
}

// ------------------------------------------------------- linear part

// The linear part of F_j on the matrix cores. For element j and shift k the
// right sum takes beta_k s_{j+k} (j+k < L) and the left sum beta_k s_{j-k}
// (j-k >= 0), beta_k = B_k where the chunk of k is covered for j's 64-element
// block (split_block_bound) and B'_k elsewhere. Elements come in groups of 32
// (group G: j = 32 G + a) and shifts in chunks of 32 (chunk c: k = 32 c + 1 +
// kappa). For group G and chunk c the +-1 factors form a 32 x 32 matrix that
// depends on G + c only on the right (entry (a, kappa) is s at position
// 32 (G + c) + 1 + a + kappa: Hankel) and on G - c only on the left (position
// 32 (G - c) - 1 + a - kappa: Toeplitz); positions outside 0..L-1 are 0.
//
// One v_mfma_i32_32x32x32_i8 multiplies such a matrix by 32 columns: 4
// column sets x of the 8 signed byte digits of beta over one chunk each. A
// wavefront owns 1024 elements (32 groups from G_w) in 8 accumulators:
// accumulator b holds groups G_w + b + 8x, x = 0..3. On the right, the digit
// tile of step c0 holds chunks c0 - 8x; accumulator b multiplies it by the
// matrix of index c0 + G_w + b, which serves all four of its column sets. So
// one tile load feeds 8 products, and consecutive steps share 7 of their 8
// matrices (each step expands one new one from the sequence bits). The left
// side runs the same way with chunks c0 + 8x and matrix index G_w + b - c0.
// The int32 sums per digit (at most 128 (L-1) in magnitude per side) are
// combined per element into the sum in units of U.
//
// Work item: (walk, 4096-element block q, k-split); a block of four
// wavefronts, wavefront x taking elements 4096 q' + 1024 x .. + 1023, q' being
// the block q positions past the one holding the neighbourhood's first
// element. Items for the whole batch are laid out so that one walk's items run
// on one XCD (workgroup i goes to XCD i mod 8), keeping its digits in that
// XCD's L2; padding items carry walk kLinNoWalk.
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef unsigned v2u __attribute__((ext_vector_type(2)));

constexpr int kLinWaves = kLinBlockElems / kLinWaveElems;
constexpr int kLinAcc = 8;                       // accumulators per wavefront
constexpr int kLinPrefetch = 3;                  // steps between a load and its use
static_assert(kLinWaveElems == 32 * 4 * kLinAcc, "a wavefront's groups are its accumulators' column sets");

__device__ __forceinline__ v4i ldg_v4i(const int8_t *p)
{
    return *(const __attribute__((address_space(1))) v4i *)(p);
}

__device__ __forceinline__ v2u ldg_v2u(const uint32_t *p)
{
    return *(const __attribute__((address_space(1))) v2u *)(p);
}

// Per-lane constants of k_lin. Operand layout of v_mfma_i32_32x32x32_i8:
// lane l holds row (A) or column (B) l % 32 and the 16 bytes k = 16 (l / 32)
// .. +15 of it.
struct LinLane {
    int x;                  // B: column set (column = 8 x + digit)
    uint32_t off0, off1;    // B: byte offset of this lane's digit row in set 0 / set 1, plus its 16 k-bytes
    uint32_t offz;          // B: the same in the zero chunk
    int n[4];               // covered chunks (c < n) of the column set's four 64-element blocks
    int lo, hi;             // min and max of n
    int pb;                 // A: position of this lane's first entry is 32 (matrix index) + pb
    int woff;               // A: first sequence word = matrix index + woff
    uint32_t sh;            // A: bit offset in it
};

// The 32 x 32 +-1 matrix of index idx, this lane's 16 entries: bytes 0x01
// (+1) and 0xFF (-1) from the sequence bits wv via a byte table (entry e:
// byte t is -1 where bit t of e is set), 0 at positions outside 0..L-1 (only
// matrices at the ends of the sequence have such entries: `edge`).
template <bool RIGHT>
__device__ __forceinline__ v4i lin_matrix(v2u wv, int idx, const LinLane &ln, int L,
                                          const v2u *__restrict__ lut)
{
    const uint32_t y = __builtin_amdgcn_alignbit(wv.y, wv.x, ln.sh);
    const uint32_t x = RIGHT ? y : __builtin_bitreverse32(y) >> 16;   // bit t: entry t
    const v2u e0 = lut[x & 0xFFu], e1 = lut[(x >> 8) & 0xFFu];
    v4i r = {(int)e0.x, (int)e0.y, (int)e1.x, (int)e1.y};
    // right: entries t at P + t (< L needed; P >= 1); left: at P - t (>= 0
    // needed; P - t <= L - 2 for every real element)
    const bool edge = RIGHT ? 32 * idx + 63 >= L : idx <= 0;
    if (edge) {
        const int P = 32 * idx + ln.pb;
        const int valid = RIGHT ? L - P : P + 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int nv = min(4, max(0, valid - 4 * q));
            const uint32_t m = nv >= 4 ? 0xFFFFFFFFu : ((1u << (8 * nv)) - 1u);
            r[q] = (int)((uint32_t)r[q] & m);
        }
    }
    return r;
}

__device__ __forceinline__ int lin_wave_min(int v)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) v = min(v, __shfl_xor(v, d));
    return v;
}

__device__ __forceinline__ int lin_wave_max(int v)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) v = max(v, __shfl_xor(v, d));
    return v;
}

// One side's products into acc over tiles c0 = cs .. ce-1. The main loop runs
// whole 9-step rounds (the steps past ce multiply zero tiles or zero
// matrices) and leaves out every lane's mixed chunks (those whose column
// set's blocks disagree on coverage); a second pass visits the steps where
// some lane's chunk is mixed and adds those products with the tile of each
// block pair. The two passes add disjoint terms of the same sums.
template <bool RIGHT>
__device__ __forceinline__ void lin_side(v16i (&acc)[kLinAcc], const LinLane &ln,
                                         const uint32_t *__restrict__ w32, const int8_t *__restrict__ limbs,
                                         const v2u *__restrict__ lut, int L, int Gw, int c_lo, int c_hi, int cs,
                                         int ce)
{
    // matrix index of accumulator b at step c0; the step's new matrix is that
    // of accumulator kFresh
    constexpr int kFresh = RIGHT ? kLinAcc - 1 : 0;
    auto midx = [&](int c0, int b) { return RIGHT ? c0 + Gw + b : Gw + b - c0; };
    auto chunk = [&](int c0) { return RIGHT ? c0 - 8 * ln.x : c0 + 8 * ln.x; };
    // w32 points 32 words before the sequence (every index here is above -32)
    auto fetch = [&](int idx) { return ldg_v2u(w32 + (uint32_t)(idx + ln.woff + 32)); };
    // (bitwise, not short-circuit, so that the lane predicates stay selects)
    auto in_range = [&](int c) { return (uint32_t)(c - c_lo) < (uint32_t)(c_hi - c_lo); };
    auto mixed = [&](int c) { return (c >= ln.lo) & (c < ln.hi) & in_range(c); };
    // this lane's 16 digit bytes of chunk c (the zero chunk unless `take`)
    auto tile = [&](int c, bool take, bool set1) {
        const uint32_t off = take ? (set1 ? ln.off1 : ln.off0) + 32u * (uint32_t)c : ln.offz;
        return ldg_v4i(limbs + off);
    };
    auto tile_main = [&](int c) { return tile(c, in_range(c) & ((c < ln.lo) | (c >= ln.hi)), c < ln.lo); };
    // Matrices in a ring of kRing = 9 slots: the matrix of accumulator b at
    // step cs + v sits in slot (v + b) % 9 on the right and (v + 7 - b) % 9 on
    // the left, so step v uses slots v .. v+7 and the matrix new at step v+1
    // (slot (v + 8) % 9) is expanded during step v's products. The sequence
    // words of that matrix and the digit tiles are loaded kLinPrefetch steps
    // before their use.
    constexpr int kRing = kLinAcc + 1;
    static_assert(kRing % kLinPrefetch == 0, "the unrolled round holds whole prefetch cycles");
    v4i A[kRing];
    {
        v2u pw[kLinAcc];                        // all loads issued before the first use
#pragma unroll
        for (int b = 0; b < kLinAcc; ++b) pw[b] = fetch(midx(cs, b));
#pragma unroll
        for (int b = 0; b < kLinAcc; ++b)
            A[RIGHT ? b : kLinAcc - 1 - b] = lin_matrix<RIGHT>(pw[b], midx(cs, b), ln, L, lut);
    }
    // wq[k % P]: words of the new matrix of step k (k >= 1); tq[k % P]: tile of step k
    v2u wq[kLinPrefetch];
    v4i tq[kLinPrefetch];
#pragma unroll
    for (int p = 0; p < kLinPrefetch; ++p) {
        wq[(p + 1) % kLinPrefetch] = fetch(midx(cs + p + 1, kFresh));
        tq[p] = tile_main(chunk(cs + p));
    }
    for (int c0b = cs; c0b < ce; c0b += kRing) {
#pragma unroll
        for (int v = 0; v < kRing; ++v) {
            const int c0 = c0b + v;
            const v4i T = tq[v % kLinPrefetch];
            tq[v % kLinPrefetch] = tile_main(chunk(c0 + kLinPrefetch));
            const v2u wn = wq[(v + 1) % kLinPrefetch];
            wq[(v + 1) % kLinPrefetch] = fetch(midx(c0 + 1 + kLinPrefetch, kFresh));
#pragma unroll
            for (int b = 0; b < kLinAcc; ++b) {
                const int slot = RIGHT ? (v + b) % kRing : (v + kLinAcc - 1 - b) % kRing;
                acc[b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[slot], T, acc[b], 0, 0, 0);
            }
            A[(v + kLinAcc) % kRing] = lin_matrix<RIGHT>(wn, midx(c0 + 1, kFresh), ln, L, lut);
        }
    }
    // mixed chunks: lane chunk c in [lo, hi) at steps c0 = c +- 8x. The steps
    // with a mixed lane are marked in 64-step masks first; each such step then
    // issues all its loads (the 8 matrices' sequence words and the 4 block
    // pairs' tiles) before it waits, and adds its 8 products.
    const bool has = ln.lo < ln.hi;
    const int z_lo = RIGHT ? ln.lo + 8 * ln.x : ln.lo - 8 * ln.x;
    const int z0 = max(cs, lin_wave_min(has ? z_lo : INT_MAX));
    const int z1 = min(ce, lin_wave_max(has ? z_lo + (ln.hi - ln.lo) : INT_MIN));
    for (int zb = z0; zb < z1; zb += 64) {
        uint64_t steps = 0;
        for (int i = 0; i < 64 && zb + i < z1; ++i)
            if (__any(mixed(chunk(zb + i)))) steps |= 1ull << i;
        while (steps) {
            const int c0 = zb + __builtin_ctzll(steps);
            steps &= steps - 1;
            const int c = chunk(c0);
            const bool mx = mixed(c);
            v2u wv[kLinAcc];
            v4i T[4];
#pragma unroll
            for (int b = 0; b < kLinAcc; ++b) wv[b] = fetch(midx(c0, b));
#pragma unroll
            for (int p = 0; p < 4; ++p) T[p] = tile(c, mx, c < ln.n[p]);
#pragma unroll
            for (int b = 0; b < kLinAcc; ++b) {
                const v4i Am = lin_matrix<RIGHT>(wv[b], midx(c0, b), ln, L, lut);
                acc[b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Am, T[b / 2], acc[b], 0, 0, 0);
            }
        }
    }
}

__global__ __launch_bounds__(64 * kLinWaves) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_lin(
    const WalkDev *__restrict__ walks, const BatchEntry *__restrict__ batch, const EvalItem *__restrict__ items)
{
    __shared__ v2u s_lut[256];
    const EvalItem it = items[blockIdx.x];
    {
        const uint32_t e = threadIdx.x;         // 256 threads, one entry each
        uint32_t lo = 0, hi = 0;
        for (int t = 0; t < 4; ++t) {
            lo |= (((e >> t) & 1u) ? 0xFFu : 0x01u) << (8 * t);
            hi |= (((e >> (t + 4)) & 1u) ? 0xFFu : 0x01u) << (8 * t);
        }
        s_lut[e] = v2u{lo, hi};
    }
    __syncthreads();
    // no barrier from here on: wavefronts leave independently
    if (it.walk == kLinNoWalk) return;
    const BatchEntry be = batch[it.walk];
    if (!be.lsplit || !be.ss->use) return;
    const WalkDev &w = walks[be.slot];
    const int L = (int)w.L;
    const uint32_t start = be.fixed ? be.start : step_start(w);
    // the sequence words from 32 words before the first (the guard words
    // before it are zero and at least 2 nw + 4 >= 68 when L >= 2048)
    const uint32_t *__restrict__ w32 = reinterpret_cast<const uint32_t *>(w.pivot) - 32;
    const int nchunks = (L - 1 + 31) / 32;
    const uint32_t K = split_row((uint32_t)L);
    const int nblk = (L + kLinBlockElems - 1) / kLinBlockElems;
    const int first = (int)(((start + 1u) % (uint32_t)L) / kLinBlockElems);
    const int blk = (first + (int)it.tile) % nblk;
    const int per = (nchunks + (int)be.lsplit - 1) / (int)be.lsplit;
    const int c_lo = (int)it.ks * per, c_hi = min(nchunks, c_lo + per);
    // the wavefront index read as a scalar: every matrix index, chunk bound
    // and end-of-sequence test below is then uniform
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = (int)threadIdx.x & 63;
    const int jw = kLinBlockElems * blk + kLinWaveElems * wave;
    if (jw >= L) return;
    const int Gw = jw >> 5;
    const int h = lane >> 5, row = lane & 31, dig = lane & 7;

    LinLane ln;
    ln.x = (lane & 31) >> 3;
    ln.off0 = (uint32_t)dig * K + 16u * (uint32_t)h;
    ln.off1 = (uint32_t)(kLimbs + dig) * K + 16u * (uint32_t)h;
    ln.offz = ln.off0 + 32u * (uint32_t)nchunks;
    ln.lo = INT_MAX;
    ln.hi = INT_MIN;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        ln.n[p] = split_block_bound(min(jw + 256 * ln.x + 64 * p, L - 1), L) >> 5;
        ln.lo = min(ln.lo, ln.n[p]);
        ln.hi = max(ln.hi, ln.n[p]);
    }
    v16i acc[kLinAcc];
#pragma unroll
    for (int b = 0; b < kLinAcc; ++b) acc[b] = v16i{};
    if (c_lo < c_hi) {
        // right: position 32 t + 1 + row + 16 h for entries of matrix index t
        const int tmax = (L - 2) >> 5;                   // the last index with a position below L
        {
            const int r0 = 1 + row + 16 * h;
            ln.pb = r0;
            ln.woff = r0 >> 5;
            ln.sh = (uint32_t)r0 & 31u;
            const int cs = c_lo, ce = min(c_hi + 24, tmax - Gw + 1);
            if (cs < ce) lin_side<true>(acc, ln, w32, be.limbs, s_lut, L, Gw, c_lo, c_hi, cs, ce);
        }
        // left: entries t = 0..15 at positions P - t, P = 32 u - 1 + row - 16 h,
        // read as the 32 bits from P - 15 on
        {
            const int q0 = row - 16 - 16 * h;
            ln.pb = q0 + 15;
            ln.woff = q0 >> 5;                           // arithmetic shift: floor
            ln.sh = (uint32_t)q0 & 31u;
            const int cs = c_lo - 24, ce = min(c_hi, Gw + kLinAcc);
            if (cs < ce) lin_side<false>(acc, ln, w32, be.limbs, s_lut, L, Gw, c_lo, c_hi, cs, ce);
        }
    }
    // accumulator b, register r: row (r % 4) + 8 (r / 4) + 4 h of group
    // G_w + b + 8 x, digit `dig`; the eight digits of an element sit in eight
    // consecutive lanes
    double *__restrict__ out = be.lpart + (size_t)it.ks * L;
#pragma unroll
    for (int b = 0; b < kLinAcc; ++b) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            double v = ldexp((double)acc[b][r], 8 * dig);
            v += __shfl_xor(v, 1);
            v += __shfl_xor(v, 2);
            v += __shfl_xor(v, 4);
            const int j = 32 * (Gw + b + 8 * ln.x) + (r & 3) + 8 * (r >> 2) + 4 * h;
            if (dig == 0 && j < L) out[j] = v;
        }
    }
}

hipError_t launch_lin(const WalkDev *walks, const BatchEntry *batch, const EvalItem *items, uint32_t n_items,
                      hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    k_lin<<<n_items, 64 * kLinWaves, 0, s>>>(walks, batch, items);
    return hipGetLastError();
}

}  // namespace psl
