// psl_eval.hip -- the neighbourhood evaluation of libpsl (gfx950): the hot
// path of Algorithm 1's Neighborhood call. For every candidate flip j and
// every shift k the one-element flip of Section 3 gives
// C'_k = C_k - 2 s_j (s_{j+k}[j+k<L] + s_{j-k}[j-k>=0]) (with Eq. (2)); from
// the C'_k the kernel accumulates F_j = sum_k |C'_k|^alpha (Eq. (5)) and
// PSL_j = max_k |C'_k| (Eq. (3)).
//
// Layout: one lane per candidate, 64 candidates per wavefront, 4, 8 or 16
// wavefronts per block; shifts are swept in LDS-staged tiles (see eval_item),
// one block per work item or a persistent grid over per-XCD queues.
#include "psl_dev_util.h"
#include "psl_device.h"
#include "psl_launch.h"

#include <algorithm>
#include <climits>

namespace psl {

// Wave-wide minimum / maximum of an int (result uniform; every lane of the
// wavefront active). lane = this lane's index in its wavefront, passed in
// so that the permute addresses derive from the caller's value.
__device__ __forceinline__ int wave_min(int v, int lane)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, __builtin_amdgcn_ds_bpermute((lane ^ o) << 2, v));
    return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ int wave_max(int v, int lane)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __builtin_amdgcn_ds_bpermute((lane ^ o) << 2, v));
    return __builtin_amdgcn_readfirstlane(v);
}

// One-neighbour tables of a 32-shift window: eight quads of shifts, 16
// entries each, indexed by the quad's four bits.
constexpr int kOneQuads = 8;
constexpr int kOneWin = 16 * kOneQuads;
constexpr int kOneItems = 4 * kOneQuads;   // table-building items per window

// Shifts per LDS tile of the table form: 256 for blocks of 8 and 16
// wavefronts (whose registers admit three and two blocks per CU whatever
// their LDS), 128 for blocks of 4, whose LDS then admits six blocks per CU.
// The split form keeps tiles of kTileK shifts in the same arrays.
template <int WAVES>
constexpr int kTabTileK = WAVES >= 8 ? kTileK : kTileK / 2;

constexpr int lds_max(int a, int b) { return a > b ? a : b; }

// LDS of one evaluation block.
template <int WAVES>
struct EvalLds {
    static constexpr int TK = kTabTileK<WAVES>;
    // first, so that a window's two-word read needs no base offset (the
    // offsets of ds_read2_b32 are 8-bit dword counts)
    uint32_t bits[WAVES * 64];          // per wavefront: its pivot words of the tile
    // table form: T(|C_k + 2m|), m = -2..2, per shift; split form: D_k and
    // B_k - B'_k per shift
    double rows[lds_max(TK * kRowStride, 2 * kTileK)];
    // table form: pair sums, both neighbours; split form: the D quad tables
    double both[lds_max(TK / 2 * 16, kChunks * kOneWin)];
    double one[TK / 32 * kOneWin];      // quad sums, one neighbour
    uint32_t both_max[TK / 2 * 16];     // max hi32 of the pair (dense PSL only)
    uint32_t one_max[TK / 32 * kOneWin];
    int kend[WAVES];                    // per wavefront
    int bmax[WAVES];
    int omax[WAVES];
};

// The sweep of one item. kMax: keep the PSL maximum in the main loop (dense
// form); otherwise the near-peak pass supplies it.
template <int WAVES, bool kMax>
__device__ __forceinline__ void eval_sweep(EvalLds<WAVES> &sh, const WalkDev &w, const BatchEntry &be,
                                           const EvalItem &it, const double *__restrict__ T,
                                           uint32_t n_lmt, int j, uint32_t SJ, int k_lo, int k_hi,
                                           int tid, double &sum, double &comp, uint32_t &mx)
{
    constexpr int TK = kTabTileK<WAVES>, TC = TK / 32, TP = TK / 2;
    const int L = (int)w.L;
    const int32_t *__restrict__ C = w.C;
    const uint32_t *__restrict__ w32 = reinterpret_cast<const uint32_t *>(w.pivot);

    // in-bounds limits: right neighbour for k <= jr, left for k <= jl
    const int jl = j, jr = L - 1 - j;
    const int lane = tid & 63;
    const int jl_min = wave_min(jl, lane), jl_max = wave_max(jl, lane);
    const int jr_min = wave_min(jr, lane), jr_max = wave_max(jr, lane);
    const int both_max = min(jl_min, jr_min);             // all lanes: both exist
    const int one_max = max(jl_min, jr_min);              // all lanes: one exists
    // first shift at which every lane of the wave has neither neighbour,
    // rounded up to a chunk start; explicit shifts end there
    const int k_none = max(jl_max, jr_max) + 1;
    const int k_wend = min(k_hi, 1 + 32 * ((k_none - 1 + 31) / 32));
    const int wave = tid >> 6;
    if ((tid & 63) == 0) {
        sh.kend[wave] = k_wend;
        sh.bmax[wave] = both_max;
        sh.omax[wave] = one_max;
    }
    __syncthreads();
    int k_bend = sh.kend[0], b_bmax = sh.bmax[0], b_omax = sh.omax[0];
    for (int x = 1; x < WAVES; ++x) {
        k_bend = max(k_bend, sh.kend[x]);
        b_bmax = max(b_bmax, sh.bmax[x]);
        b_omax = max(b_omax, sh.omax[x]);
    }

    // bit windows: the right window of chunk c starts at element
    // j + 1 + 32c (words (j+1)/32 + c and the next, shift (j+1)%32); the
    // left window ends at element j - 1 - 32c and starts at j - 32 - 32c
    // (words j/32 - 1 - c and the next, shift j%32). Per tile each
    // wavefront stages the words its windows read in LDS: the lanes of a
    // wavefront hold consecutive scan indices, so their j form at most two
    // runs of consecutive values (two when the scan wraps past L-1); per run
    // g, 16 slots of right words in increasing order and 16 slots of left
    // words in decreasing order.
    const uint32_t sh_r = (uint32_t)(j + 1) & 31u;
    const uint32_t sh_l = (uint32_t)j & 31u;
    const int j_first = __builtin_amdgcn_readlane(j, 0);
    const int grp = j < j_first ? 1 : 0;
    constexpr int kNone = 1 << 30;                        // empty run: min > max
    const int jmn0 = wave_min(grp ? kNone : j, lane), jmx0 = wave_max(grp ? -kNone : j, lane);
    const int jmn1 = wave_min(grp ? j : kNone, lane), jmx1 = wave_max(grp ? j : -kNone, lane);
    const int jmn = grp ? jmn1 : jmn0, jmx = grp ? jmx1 : jmx0;
    const uint32_t *rbits = sh.bits + 64 * wave + 32 * grp + (((j + 1) >> 5) - ((jmn + 1) >> 5));
    const uint32_t *lbits = sh.bits + 64 * wave + 32 * grp + 16 + ((jmx >> 5) - (j >> 5));
    // the slots this lane stages: run lane/32, side (lane/16)%2, slot lane%16
    const int s_grp = lane >> 5, s_side = (lane >> 4) & 1, s_idx = lane & 15;
    const int s_mn = s_grp ? jmn1 : jmn0, s_mx = s_grp ? jmx1 : jmx0;
    const int s_span = s_side ? (s_mx >> 5) - (s_mn >> 5) : ((s_mx + 1) >> 5) - ((s_mn + 1) >> 5);

    for (int kt = k_lo; kt < k_bend; kt += TK) {
        const int kt_end = min(k_bend, kt + TK);
        const int nt = kt_end - kt;
        // which pair tables some wave of the block can use in this tile
        const bool need_both = kt + 31 <= b_bmax;
        const bool need_one = kt + 31 <= b_omax;
        __syncthreads();
        {
            // this wavefront's words for its windows of the tile (chunks
            // cb .. cb + cc_last)
            const int cb = (kt - 1) >> 5;
            const int cc_last = kt < k_wend ? min(TC - 1, (k_wend - 1 - kt) >> 5) : -1;
            if (s_mn <= s_mx && s_idx < s_span + cc_last + 2) {
                const int word = s_side ? (s_mx >> 5) - cb - s_idx : ((s_mn + 1) >> 5) + cb + s_idx;
                sh.bits[64 * wave + lane] = w32[word];
            }
        }
        for (int t = tid; t < nt; t += 64 * WAVES) {
            const int c = C[kt + t];
#pragma unroll
            for (int m = 0; m < kRowStride; ++m) {
                int a = c + 2 * m - 4;
                a = a < 0 ? -a : a;
                sh.rows[t * kRowStride + m] = T[a];
            }
        }
        __syncthreads();
        if (need_both) {
            // both neighbours: C' = C + 4(xr + xl - 1), row entry 2(xr + xl).
            // Entry x of pair p: low two bits the left pair (xl_k, xl_k+1),
            // high two the right pair; one thread per (pair, right bits)
            // writes its four consecutive entries.
            for (int e = tid; e < TP * 4; e += 64 * WAVES) {
                const int p = e >> 2, r0 = e & 1, r1 = (e >> 1) & 1;
                if (2 * p + 1 < nt) {
                    const double *ra = sh.rows + (2 * p) * kRowStride + 2 * r0;
                    const double *rb = sh.rows + (2 * p + 1) * kRowStride + 2 * r1;
                    const double a0 = ra[0], a1 = ra[2], b0 = rb[0], b1 = rb[2];
                    double2 *dst = reinterpret_cast<double2 *>(sh.both + 4 * e);
                    dst[0] = make_double2(a0 + b0, a1 + b0);
                    dst[1] = make_double2(a0 + b1, a1 + b1);
                    if (kMax) {
                        const uint32_t ha0 = hi32(a0), ha1 = hi32(a1), hb0 = hi32(b0), hb1 = hi32(b1);
                        *reinterpret_cast<uint4 *>(sh.both_max + 4 * e) =
                            make_uint4(max(ha0, hb0), max(ha1, hb0), max(ha0, hb1), max(ha1, hb1));
                    }
                }
            }
        }
        if (need_one) {
            // one neighbour: C' = C + 2(2x - 1), row entry 1 + 2x. Entry x of
            // quad q: bit i of x is the bit of shift 4q + i. Item (q, h) of a
            // window writes the four consecutive entries whose two high bits
            // are h: (a + b) + (c + d).
            for (int f = tid; f < TC * kOneItems; f += 64 * WAVES) {
                const int cc = f / kOneItems, r = f - cc * kOneItems;
                const int q = r >> 2, h0 = r & 1, h1 = (r >> 1) & 1;
                const int t0 = 32 * cc + 4 * q;
                if (t0 + 3 < nt) {
                    const double *ra = sh.rows + t0 * kRowStride + 1;
                    const double a0 = ra[0], a1 = ra[2];
                    const double b0 = ra[kRowStride], b1 = ra[kRowStride + 2];
                    const double c = ra[2 * kRowStride + 2 * h0], d = ra[3 * kRowStride + 2 * h1];
                    const double cd = c + d;
                    double2 *dst = reinterpret_cast<double2 *>(sh.one + kOneWin * cc + 16 * q + 4 * (r & 3));
                    dst[0] = make_double2((a0 + b0) + cd, (a1 + b0) + cd);
                    dst[1] = make_double2((a0 + b1) + cd, (a1 + b1) + cd);
                    if (kMax) {
                        const uint32_t hcd = max(hi32(c), hi32(d));
                        const uint32_t ha0 = max(hi32(a0), hcd), ha1 = max(hi32(a1), hcd);
                        const uint32_t hb0 = hi32(b0), hb1 = hi32(b1);
                        *reinterpret_cast<uint4 *>(sh.one_max + kOneWin * cc + 16 * q + 4 * (r & 3)) =
                            make_uint4(max(ha0, hb0), max(ha1, hb0), max(ha0, hb1), max(ha1, hb1));
                    }
                }
            }
        }
        __syncthreads();

        double acc = 0.0;
        // the next window's words are read one window ahead (slots past
        // the staged ones hold stale words that are never used)
        uint32_t r0 = rbits[0], r1 = rbits[1], l0 = lbits[0], l1 = lbits[1];
#pragma unroll
        for (int cc = 0; cc < TC; ++cc) {
            const int k0 = kt + 32 * cc;
            const uint32_t cr0 = r0, cr1 = r1, cl0 = l0, cl1 = l1;
            if (cc + 1 < TC) {
                r0 = rbits[cc + 1];
                r1 = rbits[cc + 2];
                l0 = lbits[cc + 1];
                l1 = lbits[cc + 2];
            }
            if (k0 < k_wend) {
                // a side's window bits, x = 1 where s_j times the neighbour is
                // -1 (formed only in the forms that use that side)
                auto win_r = [&]() { return __builtin_amdgcn_alignbit(cr1, cr0, sh_r) ^ SJ; };
                auto win_l = [&]() {
                    return __builtin_bitreverse32(__builtin_amdgcn_alignbit(cl0, cl1, sh_l) ^ SJ);
                };
                const int tcount = min(32, kt_end - k0);
                const double *bp = sh.both + (16 * 16) * cc;
                const double *op = sh.one + kOneWin * cc;
                const uint32_t *bq = sh.both_max + (16 * 16) * cc;
                const uint32_t *oq = sh.one_max + kOneWin * cc;
                if (tcount == 32 && k0 + 31 <= both_max) {
                    const uint32_t XR = win_r(), XL = win_l();
                    // nibble q of W0 (W1) is the table index of pair 2q
                    // (2q+1): its two left bits below its two right bits
                    const uint32_t W0 = (XL & 0x33333333u) | ((XR << 2) & 0xCCCCCCCCu);
                    const uint32_t W1 = ((XL >> 2) & 0x33333333u) | (XR & 0xCCCCCCCCu);
                    // the reads go out in groups of eight before their adds
#pragma unroll
                    for (int h = 0; h < 16; h += 8) {
                        double v[8];
#pragma unroll
                        for (int p = h; p < h + 8; ++p) {
                            const uint32_t x = ((p & 1 ? W1 : W0) >> (4 * (p >> 1))) & 15u;
                            v[p - h] = bp[16 * p + x];
                            if (kMax) mx = max(mx, bq[16 * p + x]);
                        }
#pragma unroll
                        for (int p = 0; p < 8; ++p) acc += v[p];
                    }
                } else if (tcount == 32 && k0 + 31 <= jr_min && k0 > jl_max) {
                    const uint32_t XR = win_r();
                    double v[kOneQuads];
#pragma unroll
                    for (int q = 0; q < kOneQuads; ++q) {
                        const uint32_t x = (XR >> (4 * q)) & 15u;
                        v[q] = op[16 * q + x];
                        if (kMax) mx = max(mx, oq[16 * q + x]);
                    }
#pragma unroll
                    for (int q = 0; q < kOneQuads; ++q) acc += v[q];
                } else if (tcount == 32 && k0 + 31 <= jl_min && k0 > jr_max) {
                    const uint32_t XL = win_l();
                    double v[kOneQuads];
#pragma unroll
                    for (int q = 0; q < kOneQuads; ++q) {
                        const uint32_t x = (XL >> (4 * q)) & 15u;
                        v[q] = op[16 * q + x];
                        if (kMax) mx = max(mx, oq[16 * q + x]);
                    }
#pragma unroll
                    for (int q = 0; q < kOneQuads; ++q) acc += v[q];
                } else {
                    // mixed bounds or a partial chunk: per shift
                    const uint32_t XR = win_r(), XL = win_l();
                    const double *rb = sh.rows + (32 * cc) * kRowStride;
                    for (int t = 0; t < tcount; ++t) {
                        const int k = k0 + t;
                        int m = 2;
                        if (k <= jr) m += ((XR >> t) & 1u) ? 1 : -1;
                        if (k <= jl) m += ((XL >> t) & 1u) ? 1 : -1;
                        const double v = rb[t * kRowStride + m];
                        acc += v;
                        if (kMax) mx = max(mx, hi32(v));
                    }
                }
            }
        }
        nsum_add(sum, comp, acc);
    }
    // shifts where no lane of the wave has a neighbour in bounds (kn is a
    // chunk start; k_hi a chunk start or L): C'_k = C_k there. Blocks of 16
    // wavefronts take their terms and PSL part from the suffix arrays (the
    // step's launch_suffix scans the chunk values for them, the chunk arrays'
    // last entry terminating); smaller blocks add the chunk sums [xa, xb)
    // themselves (positive values; lane l takes chunks xa + l, xa + l + 64,
    // ... in order, then a fixed butterfly; every lane ends with the same sum)
    // and take the chunks' largest |C_k|.
    const int kn = max(k_lo, k_wend);
    if (kn < k_hi) {
        const int nchunks = (L - 1 + 31) / 32;
        const int xa = (kn - 1) >> 5;
        const int xb = k_hi >= L ? nchunks : (k_hi - 1) >> 5;
        if constexpr (WAVES >= 16) {
            nsum_add(sum, comp, be.S0[xa] - be.S0[xb]);
            if (kMax) mx = max(mx, hi32(T[be.M0[xa]]));
        } else {
            double cs = 0.0;
            uint32_t cm = 0;
            for (int x = xa + lane; x < xb; x += 64) {
                cs += be.S0[x];
                if (kMax) cm = max(cm, be.M0[x]);
            }
            for (int o = 32; o > 0; o >>= 1) {
                cs += __shfl_xor(cs, o);
                if (kMax) cm = max(cm, (uint32_t)__shfl_xor((int)cm, o));
            }
            nsum_add(sum, comp, cs);
            if (kMax) mx = max(mx, hi32(T[cm]));
        }
    }
}

// The VALU part of the split evaluation for one item: over the shifts where
// both neighbours of j exist (k <= min(j, L-1-j)), sum D_k ab, plus
// (B_k - B'_k)(a + b) in the chunks the linear items took with B'_k (the
// ones not covered for j's block); every other part of F_j comes from the
// prefix sums and the linear items. Per 256-shift tile the block stages D_k
// and B_k - B'_k and builds, per quad of shifts, the 16 sums
// sum_i D_{k+i} (1 - 2 y_i) indexed by the quad's bits y = xr XOR xl (ab is
// +1 where the two neighbours are equal, -1 where they differ). A window
// covered for every lane of the wavefront takes eight table reads; windows
// on the edges of the region go shift by shift.
template <int WAVES>
__device__ __forceinline__ void eval_sweep_split(EvalLds<WAVES> &sh, const WalkDev &w, const BatchEntry &be, int j,
                                                 uint32_t sjbit, int k_lo, int k_hi, int tid, double &sum,
                                                 double &comp)
{
    const int L = (int)w.L;
    const uint32_t *__restrict__ w32 = reinterpret_cast<const uint32_t *>(w.pivot);
    double *__restrict__ sdq = sh.rows;       // [kTileK][2]: D_k, B_k - B'_k
    double *__restrict__ std_ = sh.both;      // [kChunks][8 quads][16]
    const int lane = tid & 63, wave = tid >> 6;
    const int jl = j, jr = L - 1 - j;
    const int m_j = min(jl, jr);
    const int mJ = split_block_bound(j, L);
    // coverage (k0 + 31 <= mJ) is monotone in k0: a window is covered for
    // every lane exactly when it is for the wavefront's smallest bound
    const int mJw = wave_min(mJ, lane);
    // shifts past every lane's m_j hold no VALU work; the windows end at the
    // chunk that holds the wavefront's largest m_j
    const int m_w = wave_max(m_j, lane);
    const int k_wend = min(k_hi, 1 + 32 * ((m_w + 31) / 32));
    if (lane == 0) sh.kend[wave] = k_wend;
    __syncthreads();
    int k_bend = sh.kend[0];
    for (int x = 1; x < WAVES; ++x) k_bend = max(k_bend, sh.kend[x]);

    // bit windows and their LDS staging as in eval_sweep
    const uint32_t sh_r = (uint32_t)(j + 1) & 31u;
    const uint32_t sh_l = (uint32_t)j & 31u;
    const int j_first = __builtin_amdgcn_readlane(j, 0);
    const int grp = j < j_first ? 1 : 0;
    constexpr int kNone = 1 << 30;
    const int jmn0 = wave_min(grp ? kNone : j, lane), jmx0 = wave_max(grp ? -kNone : j, lane);
    const int jmn1 = wave_min(grp ? j : kNone, lane), jmx1 = wave_max(grp ? j : -kNone, lane);
    const int jmn = grp ? jmn1 : jmn0, jmx = grp ? jmx1 : jmx0;
    const uint32_t *rbits = sh.bits + 64 * wave + 32 * grp + (((j + 1) >> 5) - ((jmn + 1) >> 5));
    const uint32_t *lbits = sh.bits + 64 * wave + 32 * grp + 16 + ((jmx >> 5) - (j >> 5));
    const int s_grp = lane >> 5, s_side = (lane >> 4) & 1, s_idx = lane & 15;
    const int s_mn = s_grp ? jmn1 : jmn0, s_mx = s_grp ? jmx1 : jmx0;
    const int s_span = s_side ? (s_mx >> 5) - (s_mn >> 5) : ((s_mx + 1) >> 5) - ((s_mn + 1) >> 5);

    for (int kt = k_lo; kt < k_bend; kt += kTileK) {
        const int kt_end = min(k_bend, kt + kTileK);
        const int nt = kt_end - kt;
        __syncthreads();
        {
            const int cb = (kt - 1) >> 5;
            const int cc_last = kt < k_wend ? min(kChunks - 1, (k_wend - 1 - kt) >> 5) : -1;
            if (s_mn <= s_mx && s_idx < s_span + cc_last + 2) {
                const int word = s_side ? (s_mx >> 5) - cb - s_idx : ((s_mn + 1) >> 5) + cb + s_idx;
                sh.bits[64 * wave + lane] = w32[word];
            }
        }
        for (int t = tid; t < nt; t += 64 * WAVES) {
            const size_t k = (size_t)(kt + t);
            sdq[2 * t] = be.dq[2 * k];
            sdq[2 * t + 1] = be.dq[2 * k + 1];
        }
        __syncthreads();
        // D tables of the tile's whole quads: entry y of quad q is
        // sum_i D_{k+i} (1 - 2 y_i), the four terms added in order i = 0..3
        for (int e = tid; e < kChunks * kOneWin; e += 64 * WAVES) {
            const int t0 = 4 * (e >> 4), y = e & 15;
            if (t0 + 3 < nt) {
                double v = 0.0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const double d = sdq[2 * (t0 + i)];
                    v += (y >> i) & 1 ? -d : d;
                }
                std_[e] = v;
            }
        }
        __syncthreads();

        double acc = 0.0;
        uint32_t r0 = rbits[0], r1 = rbits[1], l0 = lbits[0], l1 = lbits[1];
#pragma unroll
        for (int cc = 0; cc < kChunks; ++cc) {
            const int k0 = kt + 32 * cc;
            const uint32_t cr0 = r0, cr1 = r1, cl0 = l0, cl1 = l1;
            if (cc + 1 < kChunks) {
                r0 = rbits[cc + 1];
                r1 = rbits[cc + 2];
                l0 = lbits[cc + 1];
                l1 = lbits[cc + 2];
            }
            if (k0 < k_wend) {
                // element bits of the two neighbours over the window: bit t
                // of XR is s_{j+k0+t} < 0, of XL is s_{j-k0-t} < 0
                const uint32_t XR = __builtin_amdgcn_alignbit(cr1, cr0, sh_r);
                const uint32_t XL = __builtin_bitreverse32(__builtin_amdgcn_alignbit(cl0, cl1, sh_l));
                const uint32_t Y = XR ^ XL;
                const int tcount = min(32, kt_end - k0);
                if (tcount == 32 && k0 + 31 <= mJw) {
                    const double *tp = std_ + kOneWin * cc;
                    // byte b of te / to holds the byte offset (8 x nibble)
                    // of nibble 2b / 2b+1 of Y, so each table address is one
                    // byte extraction; the empty asm keeps the compiler from
                    // folding the two words back into a shift and a mask per
                    // nibble
                    uint32_t te = (Y & 0x0F0F0F0Fu) << 3, to = (Y >> 1) & 0x78787878u;
                    asm("" : "+v"(te), "+v"(to));
                    const char *tb = reinterpret_cast<const char *>(tp);
                    double v[8];
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        v[2 * b] = *reinterpret_cast<const double *>(tb + 256 * b + ((te >> (8 * b)) & 0xFFu));
                        v[2 * b + 1] =
                            *reinterpret_cast<const double *>(tb + 256 * b + 128 + ((to >> (8 * b)) & 0xFFu));
                    }
#pragma unroll
                    for (int q = 0; q < 8; ++q) acc += v[q];
                } else {
                    const bool cov = k0 + 31 <= mJ;     // this lane's block took B_k for the chunk
                    const double *dp = sdq + 2 * (32 * cc);
                    for (int t = 0; t < tcount; ++t) {
                        if (k0 + t > m_j) break;
                        const uint32_t xr = (XR >> t) & 1u, xl = (XL >> t) & 1u;
                        const double d = dp[2 * t];
                        double v = (xr ^ xl) ? -d : d;
                        if (!cov) {
                            // (B - B')(a + b): a = -s_j s_{j+k} is +1 where the
                            // bits of j and j+k differ, so a + b = 2 (xr' + xl') - 2
                            // with xr' = xr XOR sjbit, xl' = xl XOR sjbit
                            const double db = dp[2 * t + 1];
                            const int na = (int)(xr ^ sjbit) + (int)(xl ^ sjbit);
                            v += db * (double)(2 * na - 2);
                        }
                        acc += v;
                    }
                }
            }
        }
        nsum_add(sum, comp, acc);
    }
}

// Neighborhood of Algorithm 1 for one (walk, 64*WAVES candidates, k-range) item.
//
// Per tile of shifts (kTabTileK) the block stages (i) per shift the five values
// T(|C_k + 2m|), m = -2..2, and (ii) tables of pre-added terms: for shifts
// where both neighbours of j exist (C' = C + 4(xr + xl - 1)), 16 entries per
// pair of shifts (k, k+1) indexed by the four bits (xl_k, xl_k+1, xr_k,
// xr_k+1); for shifts where one neighbour exists (C' = C + 2(2x - 1)), 16
// entries per quad of shifts indexed by its four bits; x = 1 when s_j times
// that neighbour is -1. A lane takes a 32-shift window of each side's bits with
// one funnel shift; per table entry it does a shift and a mask (the two
// sides' bits are first merged nibble-wise with bit-field inserts), one LDS
// read and one FP64 add. Which form a 32-shift window uses is decided once
// per wavefront from the lanes' bounds. Shifts past every lane's
// max(j, L-1-j) come from the suffix sums. The PSL comes from the near-peak
// shifts (spread over the k-splits), or, for pivots with many near-peak shifts, from
// 32-bit maxima kept in the main loop.
template <int WAVES>
__device__ __forceinline__ void eval_item(EvalLds<WAVES> &sh, const WalkDev *__restrict__ walks,
                                          const BatchEntry *__restrict__ batch, const EvalItem it,
                                          const Tables &tabs, int tid)
{
    const BatchEntry be = batch[it.walk];
    const WalkDev &w = walks[be.slot];
    const int L = (int)w.L;
    const uint32_t n_lmt = be.fixed ? be.n_lmt : w.n_lmt;
    const uint32_t start = be.fixed ? be.start : step_start(w);
    const double *__restrict__ T = tabs.T[w.alpha];
    const uint32_t *__restrict__ w32 = reinterpret_cast<const uint32_t *>(w.pivot);

    // shifts of this split, in whole 32-shift chunks from k = 1
    const int nchunks = (L - 1 + 31) / 32;
    const int per = (nchunks + (int)be.ksplit - 1) / (int)be.ksplit;
    const int c_lo = (int)it.ks * per;
    const int c_hi = min(nchunks, c_lo + per);
    const int k_lo = 1 + 32 * c_lo;
    const int k_hi = min(L, 1 + 32 * c_hi);

    // this lane's candidate; inactive lanes keep a valid j and store nothing
    const uint32_t i = it.tile * (64 * WAVES) + (uint32_t)tid;
    const bool active = i < n_lmt;
    const uint32_t ii = active ? i : n_lmt - 1;
    const int j = (int)((start + 1u + ii) % (uint32_t)L);
    const uint32_t sjbit = (w32[j >> 5] >> (j & 31)) & 1u;
    const uint32_t SJ = sjbit ? 0xFFFFFFFFu : 0u;

    double sum = 0.0, comp = 0.0;
    uint32_t mx = 0;
    const uint32_t n_near = be.near[0];
    // the split path (psl_split.hip) chose this walk for this step: the VALU
    // takes only the both-neighbour terms it leaves (its choice implies the
    // sparse PSL form)
    const bool split = be.lsplit != 0 && be.ss->use != 0;
    if (!split && n_near > be.near_lim) {
        eval_sweep<WAVES, true>(sh, w, be, it, T, n_lmt, j, SJ, k_lo, k_hi, tid, sum, comp, mx);
    } else {
        if (split)
            eval_sweep_split<WAVES>(sh, w, be, j, sjbit, k_lo, k_hi, tid, sum, comp);
        else
            eval_sweep<WAVES, false>(sh, w, be, it, T, n_lmt, j, SJ, k_lo, k_hi, tid, sum, comp, mx);
        {
            // PSL over the near-peak shifts, every candidate, all bounds
            // cases; split s takes entries s, s + ksplit, ... (the combine
            // takes the maximum over the splits)
            const int jl = j, jr = L - 1 - j;
            int peak = 0;
            for (uint32_t q = it.ks; q < n_near; q += be.ksplit) {
                const int k = (int)be.near[1 + q];
                int c = w.C[k];
                if (k <= jr) {
                    const int p = j + k;
                    c += (((w32[p >> 5] >> (p & 31)) & 1u) ^ sjbit) ? 2 : -2;
                }
                if (k <= jl) {
                    const int p = j - k;
                    c += (((w32[p >> 5] >> (p & 31)) & 1u) ^ sjbit) ? 2 : -2;
                }
                peak = max(peak, c < 0 ? -c : c);
            }
            mx = (uint32_t)peak;          // its part of the PSL (< L, far below 0x3FF00000)
        }
    }
    if (active) {
        const size_t o = (size_t)it.ks * n_lmt + i;
        be.Fpart[o] = sum + comp;
        be.Mpart[o] = mx;
    }
}

// Register budget of the evaluation kernels: the wavefronts per SIMD that
// the blocks admitted by a CU's 160 KiB of LDS hold (at most 8).
template <int WAVES>
constexpr int kEvalWavesPerEU = (160 * 1024 / (int)sizeof(EvalLds<WAVES>)) * WAVES / 4 > 8
                                    ? 8
                                    : (160 * 1024 / (int)sizeof(EvalLds<WAVES>)) * WAVES / 4;
static_assert(kEvalWavesPerEU<4> == 6 && kEvalWavesPerEU<8> == 6 && kEvalWavesPerEU<16> == 8,
              "evaluation occupancy");
static_assert(sizeof(EvalLds<4>) <= 160 * 1024 / 6, "six 4-wavefront blocks per CU");

// One block per work item; items are laid out as 8 equal-cost XCD ranges
// padded to equal length.
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(kEvalWavesPerEU<WAVES>)))
void k_eval(const WalkDev *__restrict__ walks,
                                                     const BatchEntry *__restrict__ batch,
                                                     const EvalItem *__restrict__ items, Tables tabs)
{
    __shared__ EvalLds<WAVES> sh;
    const EvalItem it = items[xcd_remap(blockIdx.x, gridDim.x)];
    if (it.walk == kNoItem) return;     // padding of an XCD's range
    eval_item<WAVES>(sh, walks, batch, it, tabs, (int)threadIdx.x);
}

// Persistent form: a fixed grid (blocks per CU x CUs) takes items from 8
// per-XCD queues, its own XCD's first (longest items first), then the
// others'. Every block leaves once all 8 queues are drained.
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(kEvalWavesPerEU<WAVES>)))
void k_eval_persistent(const WalkDev *__restrict__ walks,
                                                                const BatchEntry *__restrict__ batch,
                                                                const EvalItem *__restrict__ items,
                                                                Tables tabs, EvalQueues *queues)
{
    __shared__ EvalLds<WAVES> sh;
    __shared__ uint32_t s_item;
    uint32_t q = blockIdx.x % 8, dry = 0;
    while (dry < 8) {
        __syncthreads();                // the previous item is done with LDS
        if (threadIdx.x == 0) {
            const uint32_t idx = atomicAdd(&queues->next[q], 1u);
            s_item = idx < queues->count[q] ? queues->base[q] + idx : kNoItem;
        }
        __syncthreads();
        const uint32_t item = s_item;
        if (item == kNoItem) {
            q = (q + 1) % 8;
            ++dry;
            continue;
        }
        // the thread index, opaque to the compiler once per item: values
        // derived from it are computed per item instead of being hoisted
        // out of this loop, where they would outlive every item in scratch
        int tid = (int)threadIdx.x;
        asm volatile("" : "+v"(tid));
        __builtin_assume(tid >= 0 && tid < 64 * WAVES);
        eval_item<WAVES>(sh, walks, batch, items[item], tabs, tid);
    }
}

__global__ void k_queue_reset(EvalQueues *queues)
{
    if (threadIdx.x < 8) queues->next[threadIdx.x] = 0;
}

// ------------------------------------------------------------ launch

hipError_t launch_eval(const WalkDev *walks, const BatchEntry *batch, const EvalItem *items,
                       uint32_t n_items, const Tables &tabs, const EvalShape &shape,
                       EvalQueues *queues, hipStream_t s)
{
    if (shape.waves != 4 && shape.waves != 8 && shape.waves != 16) return hipErrorInvalidValue;
    if (shape.persistent) {
        k_queue_reset<<<1, 64, 0, s>>>(queues);
        const uint32_t grid = shape.grid;
        if (shape.waves == 4)
            k_eval_persistent<4><<<grid, 64 * 4, 0, s>>>(walks, batch, items, tabs, queues);
        else if (shape.waves == 8)
            k_eval_persistent<8><<<grid, 64 * 8, 0, s>>>(walks, batch, items, tabs, queues);
        else
            k_eval_persistent<16><<<grid, 64 * 16, 0, s>>>(walks, batch, items, tabs, queues);
    } else if (shape.waves == 4) {
        k_eval<4><<<n_items, 64 * 4, 0, s>>>(walks, batch, items, tabs);
    } else if (shape.waves == 8) {
        k_eval<8><<<n_items, 64 * 8, 0, s>>>(walks, batch, items, tabs);
    } else {
        k_eval<16><<<n_items, 64 * 16, 0, s>>>(walks, batch, items, tabs);
    }
    return hipGetLastError();
}

}  // namespace psl
