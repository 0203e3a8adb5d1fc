// y = A x over beta(r,c) on gfx950.
//
// The paper's kernel (Algorithm 1, Code 1) walks blocks one by one and
// expands each block's packed values into a SIMD register with vexpand. The
// GPU version keeps the idea -- a mask says which lanes receive the next
// packed values -- at wavefront width: the masks of 64 / (r*c) consecutive
// blocks form one 64-bit word, and lane l of a wavefront owns bit l of that
// word. The word itself is the execution mask, the rank of a set bit among
// the set bits below it (v_mbcnt) is the lane's offset into the packed
// values, and popcount(word) advances the value cursor, so one wavefront step
// is one vexpand over 64 mask bits, with contiguous (coalesced) value loads
// and no padding anywhere.
//
// Work is split into tiles of whole row intervals (the paper's static
// partition: consecutive intervals, about equal block counts, an interval is
// never split). One workgroup of W wavefronts runs one tile:
//   A. every wavefront loads the tile's mask words (<= 64), clears bits of
//      blocks outside the tile and scans their popcounts, so each word's
//      value offset is known without a sequential cursor;
//   B. the wavefronts share the words; each active lane multiplies its value
//      by x[colidx + k] and stores the product in LDS at the value's packed
//      position (compact, in value order);
//   C. one thread per (interval, block row) adds its products: for r = 1 the
//      row's products are one contiguous LDS range; for r > 1 the thread
//      walks the interval's masks and takes its row's c-bit slice of each.
// Row sums are formed in double precision for both value types and written
// once per row (no atomics), so results are deterministic.
//
// An interval with more blocks than a tile holds gets a tile of its own and
// the long path: each lane keeps a running sum for its block row over many
// words, and the sums of lanes of the same block row are combined at the end.
#include <type_traits>

#include "common.hpp"
#include "wave_common.hpp"

namespace spc {
namespace {

// One 16-byte chunk per lane from a buffer straight into LDS (no registers).
// The builtin and its LDS address space exist for the device target only;
// in the host pass, which emits no device code, the body is empty (it would
// otherwise make every function template that reaches it invalid there).
__device__ __forceinline__ void chunk_to_lds(__amdgpu_buffer_rsrc_t vr, void *lds, uint32_t voff, int soff) {
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(vr, (__attribute__((address_space(3))) void *)lds, 16, voff, soff, 0,
                                             dev::kNT);
#endif
}

using namespace dev;

constexpr int kWaves = 4;
constexpr int kThreads = kWaves * 64;
constexpr int kUnroll = 4;

struct SpmvArgs {
    const int32_t *brow;
    const int32_t *bcol;
    const uint64_t *mw;
    const void *vals;
    const void *x;
    void *y;
    const TileDesc *tiles;
    int64_t n_rows;
    int64_t nnz;
    int64_t n_blocks;
    int64_t n_cols;
    int32_t n_tiles;
    int32_t accumulate;
    int32_t xcd_remap;
    int32_t tiles_per_xcd;
};

// Bits of block slots [lo, hi) of a word (slot = RC bits).
template <int RC>
__device__ __forceinline__ uint64_t slot_bits(int lo, int hi) {
    uint64_t upto_hi = (hi * RC >= 64) ? ~0ull : ((1ull << (hi * RC)) - 1ull);
    uint64_t below_lo = (lo * RC >= 64) ? ~0ull : ((1ull << (lo * RC)) - 1ull);
    return upto_hi & ~below_lo;
}

template <class T>
__device__ __forceinline__ T ldg_nt(const T *p) {
    return __builtin_nontemporal_load(p);
}

// Lane l of the calling wavefront gets the tile's word l (global index
// w0 + l), restricted to blocks [b0, b1).
template <class Sh>
__device__ __forceinline__ uint64_t tile_word(const uint64_t *mw, int w0, int nw, int b0, int b1, int l) {
    if (l >= nw) return 0ull;
    const int gw = w0 + l;
    uint64_t m = mw[gw];
    const int lo = max(b0 - gw * Sh::BPW, 0);
    const int hi = min(b1 - gw * Sh::BPW, Sh::BPW);
    return m & slot_bits<Sh::RC>(lo, hi);
}

// ---------------------------------------------------------------------------
// Tile of whole intervals whose products fit the LDS buffer (TB values).
template <class Sh, class T, int TB>
__device__ void tile_short(const SpmvArgs &a, int i0, int i1, int b0, int b1, int64_t vbase,
                           uint64_t *s_wm, int *s_off, T *s_prod) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const T *__restrict__ vals = static_cast<const T *>(a.vals);
    const T *__restrict__ x = static_cast<const T *>(a.x);

    // A. words and their value offsets (every wavefront computes them)
    const int w0 = b0 / Sh::BPW;
    const int nw = (b1 > b0) ? ((b1 - 1) / Sh::BPW - w0 + 1) : 0;
    const uint64_t wm = tile_word<Sh>(a.mw, w0, nw, b0, b1, lane);
    const int cnt = __popcll(wm);
    const int incl = wave_incl_scan(cnt);
    const int excl = incl - cnt;
    if (wid == 0) {
        if (lane < nw) {
            s_wm[lane] = wm;
            s_off[lane] = excl;
        }
        if (lane == 0) {
            s_wm[nw] = 0ull;
            s_off[nw] = nw > 0 ? __builtin_amdgcn_readlane(incl, nw - 1) : 0;
        }
    }

    // B. products, lane = mask bit
    {
        const int slot = lane / Sh::RC;
        const int kcol = (lane % Sh::RC) % Sh::C;
        const int k0 = (nw * wid) / kWaves, k1 = (nw * (wid + 1)) / kWaves;
        for (int i = k0; i < k1; i += kUnroll) {
            uint64_t M[kUnroll];
            int off[kUnroll];
            unsigned rk[kUnroll];
            bool act[kUnroll];
            int col[kUnroll];
            T v[kUnroll], xv[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const bool in = (i + u) < k1;
                M[u] = in ? readlane64(wm, i + u) : 0ull;
                off[u] = in ? __builtin_amdgcn_readlane(excl, i + u) : 0;
                act[u] = (M[u] >> lane) & 1ull;
                rk[u] = lane_rank(M[u]);
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (act[u]) {
                    col[u] = ldg_nt(a.bcol + (int64_t)(w0 + i + u) * Sh::BPW + slot) + kcol;
                    v[u] = ldg_nt(vals + vbase + off[u] + rk[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                if (act[u]) xv[u] = x[col[u]];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                if (act[u]) s_prod[off[u] + rk[u]] = v[u] * xv[u];
        }
    }
    __syncthreads();

    // C. one thread per (interval, block row)
    T *__restrict__ y = static_cast<T *>(a.y);
    const int npairs = (i1 - i0) * Sh::R;
    for (int p = threadIdx.x; p < npairs; p += kThreads) {
        const int I = i0 + p / Sh::R;
        const int rho = p % Sh::R;
        const int bs = a.brow[I], be = a.brow[I + 1];
        double acc = 0.0;
        bool any = false;  // the row has stored entries
        if (bs < be) {
            int wi = bs / Sh::BPW - w0;
            int bit = (bs % Sh::BPW) * Sh::RC;
            int vpos = s_off[wi] + __popcll(s_wm[wi] & ((1ull << bit) - 1ull));
            if (Sh::R == 1) {
                const int we = be / Sh::BPW - w0;
                const int be_bit = (be % Sh::BPW) * Sh::RC;
                const int vend = s_off[we] + __popcll(s_wm[we] & ((1ull << be_bit) - 1ull));
                double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
                int k = vpos;
                for (; k + 4 <= vend; k += 4) {
                    a0 += (double)s_prod[k];
                    a1 += (double)s_prod[k + 1];
                    a2 += (double)s_prod[k + 2];
                    a3 += (double)s_prod[k + 3];
                }
                for (; k < vend; ++k) a0 += (double)s_prod[k];
                acc = (a0 + a1) + (a2 + a3);
                any = vend > vpos;
            } else {
                double a0 = 0.0, a1 = 0.0;
                const uint32_t below = rho ? ((1u << (rho * Sh::C)) - 1u) : 0u;
                for (int b = bs; b < be; ++b) {
                    const uint32_t m = (uint32_t)(s_wm[wi] >> bit) & Sh::RCMASK;
                    const uint32_t sub = (m >> (rho * Sh::C)) & Sh::CMASK;
                    const int pos = vpos + __popc(m & below);
                    const int n = __popc(sub);
                    any |= n > 0;
                    double part = 0.0;
                    for (int k = 0; k < n; ++k) part += (double)s_prod[pos + k];
                    if (b & 1) a1 += part; else a0 += part;
                    vpos += __popc(m);
                    bit += Sh::RC;
                    if (bit == 64) {
                        bit = 0;
                        ++wi;
                    }
                }
                acc = a0 + a1;
            }
        }
        const int64_t row = (int64_t)I * Sh::R + rho;
        if (row < a.n_rows) {
            // accumulate: a row without entries is left untouched, as the
            // paper's kernel skips empty intervals
            if (a.accumulate) {
                if (any) y[row] = (T)(acc + (double)y[row]);
            } else {
                y[row] = (T)acc;
            }
        }
    }
}


// ---------------------------------------------------------------------------
// Wavefront tiles (mode 0). A tile is small enough for one wavefront, and the
// four wavefronts of a workgroup run four independent tiles with no barrier
// between them, so a slow phase of one tile never holds up another. Per tile:
//   1. request the tile's streams at once: the packed values with 16-byte
//      loads (lane l takes chunks l, l+64, ...), the block columns, the
//      interval pointers and the mask words;
//   2. the values go to LDS in packed order; lane = mask bit then walks the
//      mask words on the scalar unit: the word is the execution mask (an
//      inverse ballot), the lane's rank among the word's set bits plus the
//      running popcount is its value's slot, and it multiplies that value by
//      x[colidx + k]; the C products of each block row are added across
//      lanes (DPP) into one partial per (block, block row), two for FP64,
//      which go to LDS;
//   3. L lanes per (interval, block row) add its partials (L as large as the
//      tile's row count allows) and combine their sums with shuffles.
template <class Sh, class T, int KQ>
struct WaveSmem {
    static constexpr int E = 16 / sizeof(T);          // values per 16-byte chunk
    static constexpr int WB = (64 * KQ - 1) * E;      // bits (so values) a tile may hold
    static constexpr int NB = WB / Sh::RC;            // blocks a tile may hold
    // NB blocks starting anywhere in a word span at most NB / BPW + 2 words
    static constexpr int NWMAX = NB / Sh::BPW + 2;
    static constexpr int NCR = (NWMAX * Sh::BPW + 63) / 64;   // 64-lane rounds of block columns
    static constexpr int NBUF = 64 * KQ * E;
    // partials per (block, block row): FP64 stops the lane sums at two per
    // block row (fewer DPP steps, each a pair of moves and an add), FP32
    // adds all C lanes (one DPP add per step)
    static constexpr int PPR = sizeof(T) == 8 ? 2 : 1;
    static constexpr int NPART = NWMAX * (64 / Sh::C) * PPR;  // partials of the tile's words
    static_assert(NPART * 8 <= NBUF * (int)sizeof(T), "the partials must fit the value buffer");
    T buf[NBUF];                                      // packed values, then the partials (double)
    // tile-relative interval pointers; they follow buf so that the value
    // reads of the last word's lanes past the tile (at most 63 entries past
    // buf, never used) stay inside this wavefront's own area
    int brow[128];
    double zero[2];                                   // read by the lanes of clear mask bits
};

// Row results of a tile held back for storing later: byte offsets into y
// (0xffffffff: nothing) and values, one per round of tile_sums.
template <class T>
struct YOut {
    uint32_t off[2];
    T val[2];
};

// 2b. Products of one mask word, added across the lanes of each block row
// down to PPR partials per (block, block row): all C lanes for FP32 (one
// partial), C/2 lanes for FP64 (two partials: columns below and from C/2).
// The lanes at column 0 (and C/2) store them at entry
// j (64 / C) PPR + lane / (C / PPR), i.e. slot j BPW + slot, block row rho,
// half h of the tile's words (slots of the next tile's blocks in the last
// word get entries that are never read). Every lane must be active.
// The lane's entry base (part + lane / W) is formed once by the caller; only
// the word's offset, a constant, is added per word. keeper: lane % W == 0.
template <class Sh, class T>
__device__ __forceinline__ void store_partial_at(double *mine, bool keeper, int j, T prod) {
    constexpr int PPR = sizeof(T) == 8 ? 2 : 1;
    constexpr int W = Sh::C / PPR;
    T p = prod;
    if constexpr (sizeof(T) == 8) {
        p += dpp_f64<0xb1>(p);                          // quad_perm [1,0,3,2]
        if constexpr (W == 4) p += dpp_f64<0x4e>(p);    // quad_perm [2,3,0,1]
    } else {
        p = row_group_sum<Sh::C>(p);
    }
    if (keeper) mine[j * (64 / Sh::C) * PPR] = (double)p;
}

// 3. Row sums of a wavefront tile whose (block, block row) partials sit in
// s_part (PPR of them at entry (g R + rho) PPR: slot g of the tile's words,
// block row rho) and whose tile-relative interval pointers sit in s_brow.
// Only the tile's own slots are read. With DEFER (and y = A x), the results
// go to *out instead of y; the caller stores them.
template <class Sh, class T, bool DEFER = false, int PPR = (sizeof(T) == 8 ? 2 : 1)>
__device__ __forceinline__ void tile_sums(const SpmvArgs &a, const TileDesc &d, int lo_slot, int w0,
                                          const int *s_brow, const double *s_part, YOut<T> *out = nullptr) {
    const int lane = threadIdx.x & 63;
    const int nI = d.i1 - d.i0;
    // L lanes per (interval, block row) add its partials. A tile has up to
    // 128 pairs: with more than 64, L = 1 and a lane takes pairs lane and
    // lane + 64.
    const int npairs = nI * Sh::R;
    // log2 L: the largest L with npairs * L <= 64
    const int lg = npairs > 64 ? 0 : npairs > 1 ? __builtin_clz((unsigned)(npairs - 1)) - 26 : 6;
    const int L = 1 << lg;
    const int l = lane & (L - 1);
    const double *__restrict__ pp = s_part;
    if (DEFER) out->off[0] = out->off[1] = 0xffffffffu;
    for (int round = 0; round < 2; ++round) {
        if (round == 1 && npairs <= 64) break;
        const int pair = (lane >> lg) + 64 * round;
        double acc = 0.0;
        bool stored = false;  // the row holds at least one entry (accumulate leaves other rows alone)
        if (pair < npairs) {
            const int li = pair / Sh::R, rho = pair % Sh::R;
            const int bs = s_brow[li], be = s_brow[li + 1];   // tile-relative blocks
            // two partials per step, so their reads share one LDS round trip
            double a0 = 0.0, a1 = 0.0;
            int b = bs + l;
            for (; b + L < be; b += 2 * L) {
                const double *e0 = pp + ((b + lo_slot) * Sh::R + rho) * PPR;
                const double *e1 = pp + ((b + L + lo_slot) * Sh::R + rho) * PPR;
#pragma unroll
                for (int h = 0; h < PPR; ++h) {
                    a0 += e0[h];
                    a1 += e1[h];
                }
            }
            if (b < be) {
                const double *e0 = pp + ((b + lo_slot) * Sh::R + rho) * PPR;
#pragma unroll
                for (int h = 0; h < PPR; ++h) a0 += e0[h];
            }
            acc = a0 + a1;
            if (Sh::R == 1) {
                stored = be > bs;  // every block holds at least one entry
            } else if (a.accumulate) {
                for (int b = bs + l; b < be; b += L) {
                    const unsigned g = (unsigned)(b + lo_slot);
                    const uint32_t m = (uint32_t)(a.mw[w0 + g / Sh::BPW] >> ((g % Sh::BPW) * Sh::RC));
                    stored = stored || ((m >> (rho * Sh::C)) & Sh::CMASK) != 0;
                }
            }
        }
        acc = group_sum(acc, lg);
        if (Sh::R > 1 && a.accumulate)
            for (int m = L >> 1; m >= 1; m >>= 1) stored = __shfl_xor((int)stored, m, 64) || stored;
        if (DEFER && !a.accumulate) {
            const int li = pair / Sh::R, rho = pair % Sh::R;
            const int64_t row = (int64_t)(d.i0 + li) * Sh::R + rho;
            const bool mine = pair < npairs && l == 0 && row < a.n_rows;
            out->off[round] = mine ? (uint32_t)row * (uint32_t)sizeof(T) : 0xffffffffu;
            out->val[round] = (T)acc;
        } else if (pair < npairs && l == 0) {
            const int li = pair / Sh::R, rho = pair % Sh::R;
            const int64_t row = (int64_t)(d.i0 + li) * Sh::R + rho;
            if (row < a.n_rows) {
                T *__restrict__ y = static_cast<T *>(a.y);
                if (a.accumulate) {
                    if (stored) y[row] = (T)(acc + (double)y[row]);
                } else {
                    y[row] = (T)acc;
                }
            }
        }
    }
}

// Stores held-back row results: always two buffer stores (an offset past
// the end stores nothing), so the count of memory operations in flight does
// not depend on the data.
template <class T>
__device__ __forceinline__ void y_flush(__amdgpu_buffer_rsrc_t yr, const YOut<T> &o) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if constexpr (sizeof(T) == 8)
            __builtin_amdgcn_raw_buffer_store_b64(
                __builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned int, (double)o.val[k]), yr, o.off[k], 0,
                0);
        else
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, (float)o.val[k]), yr, o.off[k], 0, 0);
    }
}

// Registers holding one tile's small streams while their loads are in
// flight (the packed values go straight to LDS).
template <class Sh, class T, int KQ, int NCR = WaveSmem<Sh, T, KQ>::NCR>
struct TileIn {
    int colr[NCR];   // block columns of the slots of the tile's words, 64 per register
    int br[2];   // interval pointers lane and lane + 64 (a tile has up to 127 intervals)
    uint64_t m;  // lane j: the tile's mask word j (0 past the tile's words)
};

// Issues every stream of a tile as unguarded buffer loads: the block
// columns and interval pointers into registers, then the packed values into
// LDS (s_vals, chunk k of lane l at 16 (64 k + l) bytes).
template <class Sh, class T, int KQ, int NCR>
__device__ __forceinline__ void tile_issue(const SpmvArgs &a, const TileDesc &d, TileIn<Sh, T, KQ, NCR> &in,
                                           T *s_vals) {
    using SM = WaveSmem<Sh, T, KQ>;
    constexpr int E = SM::E;
    const int lane = threadIdx.x & 63;
    const T *__restrict__ vals = static_cast<const T *>(a.vals);
    const int b0 = d.b0, b1 = d.b1, nv = d.nv, nI = d.i1 - d.i0;
    const int64_t abase = d.vbase & ~(int64_t)(E - 1);
    const int shift = (int)(d.vbase - abase);
    const int nq = (shift + nv + E - 1) / E;
    const int q_tail = (abase + (int64_t)nq * E > a.nnz) ? nq - 1 : nq;
    const int w0 = b0 / Sh::BPW;
    const int nw = (b1 > b0) ? ((b1 - 1) / Sh::BPW - w0 + 1) : 0;
    // columns of all slots of the tile's words: the blocks before b0 in the
    // first word are never used (their bits are cleared), those after b1 in
    // the last word are valid blocks of the next tile
    const int cs0 = w0 * Sh::BPW;
    const int ncs = (int)(min<int64_t>((int64_t)(w0 + nw) * Sh::BPW, a.n_blocks) - cs0);
    const auto cr = rsrc(a.bcol + cs0, (uint32_t)ncs * 4u);
#pragma unroll
    for (int k = 0; k < NCR; ++k)
        in.colr[k] = __builtin_amdgcn_raw_buffer_load_b32(cr, (uint32_t)(lane * 4), 256 * k, kNT);
    const auto brr = rsrc(a.brow + d.i0, (uint32_t)(nI + 1) * 4u);
    in.br[0] = __builtin_amdgcn_raw_buffer_load_b32(brr, (uint32_t)(lane * 4), 0, 0);
    in.br[1] = __builtin_amdgcn_raw_buffer_load_b32(brr, (uint32_t)(lane * 4), 256, 0);
    const auto mr = rsrc(a.mw + w0, (uint32_t)nw * 8u);
    in.m = __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(mr, (uint32_t)(lane * 8), 0, kNT));
    const auto vr = rsrc(vals + abase, (uint32_t)q_tail * 16u);
#pragma unroll
    for (int k = 0; k < KQ; ++k)
        chunk_to_lds(vr, s_vals + 64 * k * E, (uint32_t)(lane * 16), 1024 * k);
}

// Everything after the stream loads: the x gathers and products, the row
// sums and the y stores.
// PEND >= 0: the tile's values were loaded straight into LDS, and PEND
// vector memory operations issued after them (a next tile's streams) may
// stay in flight; PEND < 0: the values were written to LDS from registers.
template <class Sh, class T, int KQ, int PEND = 0>
__device__ void tile_run(const SpmvArgs &a, const TileDesc &d, TileIn<Sh, T, KQ> &in, __amdgpu_buffer_rsrc_t xr,
                         WaveSmem<Sh, T, KQ> &sm) {
    using SM = WaveSmem<Sh, T, KQ>;
    constexpr int E = SM::E;
    const int lane = threadIdx.x & 63;
    const T *__restrict__ vals = static_cast<const T *>(a.vals);
    const int b0 = d.b0, b1 = d.b1, nv = d.nv;
    const int64_t abase = d.vbase & ~(int64_t)(E - 1);
    const int shift = (int)(d.vbase - abase);
    const int nq = (shift + nv + E - 1) / E;          // chunks holding the tile's values
    // the array's last chunk may reach past nnz: it is read value by value
    const int q_tail = (abase + (int64_t)nq * E > a.nnz) ? nq - 1 : nq;
    const int w0 = b0 / Sh::BPW;
    const int nw = (b1 > b0) ? ((b1 - 1) / Sh::BPW - w0 + 1) : 0;
    const int lo_slot = b0 - w0 * Sh::BPW;                  // slots of word 0 before the tile
    const uint64_t lo_mask = ~low_bits(lo_slot * Sh::RC);
    // interval pointers into LDS (lanes past the tile's intervals write what
    // the out-of-range loads returned; nothing reads them)
    sm.brow[lane] = in.br[0] - b0;
    sm.brow[lane + 64] = in.br[1] - b0;
    if (lane < 2) sm.zero[lane] = 0.0;
    // 2. products, lane = mask bit, words walked on the scalar unit. Per
    // word: the lane's x gather (a lane whose bit is clear gathers out of
    // range: 0, no memory access) and its value (LDS, at the count of set bits
    // below it plus the word's running offset; zero where its bit is clear).
    // Each word's mask is used in this pass only. Once all values are read,
    // each word's products are added over each block row's C lanes and one
    // partial per (block, block row) replaces the values in LDS. The last
    // word keeps the bits of the next tile's blocks; their partials are never
    // read.
    // The gathers need only the block columns and the masks: tiles of 8
    // chunks (the most mask words) issue all of them before the wait for the
    // values, so their latency runs under the value stream's. Smaller tiles,
    // and FP32 tiles of 16- and 32-bit masks, gather word by word after the
    // wait (measured faster for them).
    constexpr bool EARLY = KQ >= 8 && (sizeof(T) == 8 || Sh::RC == 8);
    if constexpr (EARLY) {
        constexpr int NWM = SM::NWMAX;
        static_assert(NWM <= 64, "a tile's mask words fit one per lane");
        const int slot = lane / Sh::RC;
        // The NWM gathers are issued in every tile, so that the wait below counts
        // them: a tile of empty intervals has no words, its masks read as 0 (an
        // empty range) and none of its gathers touches memory.
        T xv[NWM];
        {
            const int kcol = (lane % Sh::RC) % Sh::C;
            // the column of slot j BPW + slot sits in register (j BPW) / 64 of lane
            // (j BPW + slot) mod 64 (a word's slots never straddle 64 lanes); all
            // of the tile's cross-lane moves are issued before the first is used
            int colj[NWM];
#pragma unroll
            for (int j = 0; j < NWM; ++j)
                colj[j] = __builtin_amdgcn_ds_bpermute(((j * Sh::BPW) % 64 + slot) * 4, in.colr[(j * Sh::BPW) / 64]);
#pragma unroll
            for (int j = 0; j < NWM; ++j) {
                uint64_t m = readlane64(in.m, j);
                if (j == 0) m &= lo_mask;
                xv[j] = buf_load<T>(xr, pick(m, (uint32_t)(colj[j] + kcol) * (uint32_t)sizeof(T), 0xffffffffu));
            }
        }
        // the values have landed in LDS (they were loaded before the NWM gathers
        // and the PEND later operations); the chunk reaching past nnz came back
        // as zeros and is filled value by value
        if constexpr (PEND >= 0) wait_vm_n<(PEND + NWM < 63 ? PEND + NWM : 63)>();
        if (q_tail < nq && lane < E) {
            const int64_t g = abase + (int64_t)q_tail * E + lane;
            if (g < a.nnz) sm.buf[q_tail * E + lane] = vals[g];
        }
        wave_sync();
        if (nw > 0) {
            constexpr int PPR = sizeof(T) == 8 ? 2 : 1;
            constexpr int W = Sh::C / PPR;
            const char *__restrict__ bb = reinterpret_cast<const char *>(sm.buf);
            // lanes of clear bits read a zero from LDS instead of a value
            const uint32_t zbyte = (uint32_t)(reinterpret_cast<const char *>(sm.zero) - bb);
            T pv[NWM];
            uint32_t vbyte = (uint32_t)shift * (uint32_t)sizeof(T);   // byte offset of the word's first value
#pragma unroll
            for (int j = 0; j < NWM; ++j) {
                uint64_t m = readlane64(in.m, j);
                if (j == 0) m &= lo_mask;
                pv[j] = *reinterpret_cast<const T *>(bb + pick(m, lane_rank(m) * (uint32_t)sizeof(T) + vbyte, zbyte));
                vbyte += (uint32_t)__popcll(m) * (uint32_t)sizeof(T);
            }
            wave_sync();  // all values are read before the partials overwrite them
            double *__restrict__ mine = reinterpret_cast<double *>(sm.buf) + lane / W;
            const bool keeper = (lane % W) == 0;
#pragma unroll
            for (int j = 0; j < NWM; ++j) store_partial_at<Sh, T>(mine, keeper, j, pv[j] * xv[j]);
        }
    } else {
        // the values have landed in LDS (they were loaded last); the chunk
        // reaching past nnz came back as zeros and is filled value by value
        if constexpr (PEND >= 0) wait_vm_n<PEND>();
        if (q_tail < nq && lane < E) {
            const int64_t g = abase + (int64_t)q_tail * E + lane;
            if (g < a.nnz) sm.buf[q_tail * E + lane] = vals[g];
        }
        wave_sync();

        if (nw > 0) {  // a tile of empty intervals has no words (and maybe no masks array)
            constexpr int NWM = SM::NWMAX;
            constexpr int PPR = sizeof(T) == 8 ? 2 : 1;
            constexpr int W = Sh::C / PPR;
            static_assert(NWM <= 64, "a tile's mask words fit one per lane");
            const int slot = lane / Sh::RC;
            const int kcol = (lane % Sh::RC) % Sh::C;
            const char *__restrict__ bb = reinterpret_cast<const char *>(sm.buf);
            // lanes of clear bits read a zero from LDS instead of a value
            const uint32_t zbyte = (uint32_t)(reinterpret_cast<const char *>(sm.zero) - bb);
            // the column of slot j BPW + slot sits in register (j BPW) / 64 of lane
            // (j BPW + slot) mod 64 (a word's slots never straddle 64 lanes); all
            // of the tile's cross-lane moves are issued before the first is used
            int colj[NWM];
#pragma unroll
            for (int j = 0; j < NWM; ++j)
                colj[j] = __builtin_amdgcn_ds_bpermute(((j * Sh::BPW) % 64 + slot) * 4, in.colr[(j * Sh::BPW) / 64]);
            T xv[NWM], pv[NWM];
            uint32_t vbyte = (uint32_t)shift * (uint32_t)sizeof(T);   // byte offset of the word's first value
#pragma unroll
            for (int j = 0; j < NWM; ++j) {
                uint64_t m = readlane64(in.m, j);
                if (j == 0) m &= lo_mask;
                xv[j] = buf_load<T>(xr, pick(m, (uint32_t)(colj[j] + kcol) * (uint32_t)sizeof(T), 0xffffffffu));
                pv[j] = *reinterpret_cast<const T *>(bb + pick(m, lane_rank(m) * (uint32_t)sizeof(T) + vbyte, zbyte));
                vbyte += (uint32_t)__popcll(m) * (uint32_t)sizeof(T);
            }
            wave_sync();  // all values are read before the partials overwrite them
            double *__restrict__ mine = reinterpret_cast<double *>(sm.buf) + lane / W;
            const bool keeper = (lane % W) == 0;
#pragma unroll
            for (int j = 0; j < NWM; ++j) store_partial_at<Sh, T>(mine, keeper, j, pv[j] * xv[j]);
        }
    }
    wave_sync();
    tile_sums<Sh, T>(a, d, lo_slot, w0, sm.brow, reinterpret_cast<const double *>(sm.buf));
}

template <class Sh, class T, int KQ>
__device__ __forceinline__ void wave_tile(const SpmvArgs &a, const TileDesc &d, __amdgpu_buffer_rsrc_t xr,
                                          WaveSmem<Sh, T, KQ> &sm) {
    TileIn<Sh, T, KQ> in;
    tile_issue<Sh, T, KQ>(a, d, in, sm.buf);
    tile_run<Sh, T, KQ>(a, d, in, xr, sm);
}

// ---------------------------------------------------------------------------
// Block-row lanes (mode 3). Lane (s, rho) takes block row rho of slot s of
// the tile's words and walks that block row's set bits one after another,
// gathering x at the block's column plus the bit's column; the wavefront
// takes as many steps as its fullest block row has bits, and the lane's sum
// is that block row's one partial. Where block rows hold few of their C
// entries this issues far fewer gathers than one lane per mask bit, so the
// tiles are sized by values, not by mask bits: up to the (64 KQ - 1) E
// values the LDS buffer holds, and up to NBX blocks (at most 64 mask words,
// 4032 mask bits, and partials that fit the buffer). Everything else (the
// streams, the interval pointers, the row sums) is mode 0's.
template <class Sh, class T, int KQ>
struct BrowSmem {
    using W = WaveSmem<Sh, T, KQ>;
    static constexpr int NS = 64 * Sh::BPW;              // slots of 64 mask words
    static constexpr int NSR = NS / 64;                  // 64-lane rounds over the slots
    static constexpr int NBR = NS * Sh::R / 64;          // 64-lane rounds over the block rows
    static constexpr int VCAP = (64 * KQ - 1) * W::E;    // values of a tile (any alignment fits the buffer)
    static constexpr int NPMAX = W::NBUF * (int)sizeof(T) / 8;   // partials the buffer holds
    static constexpr int NBA = 4032 / Sh::RC;
    static constexpr int NBB = NPMAX / Sh::R - Sh::BPW + 1;
    static constexpr int NBX = NBA < NBB ? NBA : NBB;   // blocks of a tile
    static_assert(NBX + Sh::BPW - 1 <= NS, "a tile's blocks fit 64 mask words");
    // per slot: mask bits (0 outside the tile's blocks) and first value, one
    // word (bits, then first << RC) where the mask has at most 16 bits
    static constexpr bool PACK = Sh::RC <= 16;
    static_assert(!PACK || VCAP < (1 << (32 - Sh::RC)), "a first value fits above the mask bits");
    using SlotT = std::conditional_t<PACK, uint32_t, uint2>;
    W w;                    // values then partials, interval pointers, zero
    SlotT slot[NS];
    __device__ __forceinline__ void put(int s, uint32_t mk, int first) {
        if constexpr (PACK) slot[s] = mk | ((uint32_t)first << Sh::RC);
        else slot[s] = make_uint2(mk, (uint32_t)first);
    }
    __device__ __forceinline__ void get(int s, uint32_t &mk, uint32_t &first) const {
        if constexpr (PACK) {
            const uint32_t e = slot[s];
            mk = e & Sh::RCMASK;
            first = e >> Sh::RC;
        } else {
            const uint2 e = slot[s];
            mk = e.x;
            first = e.y;
        }
    }
};

// Adds n products of one block row to s, in order: T = double, fused
// multiply-adds in double; T = float, products and their sum in single
// precision, as mode 0 forms them (no contraction into fused operations).
template <class T, int N>
__device__ __forceinline__ T block_row_acc(const T (&v)[N], const T (&xg)[N], int n, T s) {
#pragma unroll
    for (int it = 0; it < N; ++it) {
        if (it >= n) break;
        if constexpr (sizeof(T) == 8) s = __builtin_fma(v[it], xg[it], s);
        else s = __fadd_rn(s, __fmul_rn(v[it], xg[it]));
    }
    return s;
}

template <class Sh, class T, int KQ>
__device__ void brow_run(const SpmvArgs &a, const TileDesc &d, TileIn<Sh, T, KQ, Sh::BPW> &in,
                         __amdgpu_buffer_rsrc_t xr, BrowSmem<Sh, T, KQ> &sm) {
    using SM = BrowSmem<Sh, T, KQ>;
    constexpr int E = SM::W::E;
    constexpr int R = Sh::R, C = Sh::C, BPW = Sh::BPW;
    const int lane = threadIdx.x & 63;
    const T *__restrict__ vals = static_cast<const T *>(a.vals);
    const int b0 = d.b0, b1 = d.b1, nv = d.nv;
    const int64_t abase = d.vbase & ~(int64_t)(E - 1);
    const int shift = (int)(d.vbase - abase);
    const int nq = (shift + nv + E - 1) / E;
    const int q_tail = (abase + (int64_t)nq * E > a.nnz) ? nq - 1 : nq;
    const int w0 = b0 / BPW;
    const int lo_slot = b0 - w0 * BPW;
    const int hi_slot = lo_slot + (b1 - b0);   // the tile's blocks are slots [lo_slot, hi_slot)
    sm.w.brow[lane] = in.br[0] - b0;
    sm.w.brow[lane + 64] = in.br[1] - b0;
    if (lane < 2) sm.w.zero[lane] = 0.0;
    wait_vm_all();   // the values have landed in LDS; the chunk past nnz is filled value by value
    if (q_tail < nq && lane < E) {
        const int64_t g = abase + (int64_t)q_tail * E + lane;
        if (g < a.nnz) sm.w.buf[q_tail * E + lane] = vals[g];
    }
    if (b1 > b0) {
        // A. lane = slot: its mask bits (from the lane holding its word) and
        // its first value (a prefix over the slots' value counts)
        const int mlo = (int)(uint32_t)in.m, mhi = (int)(uint32_t)(in.m >> 32);
        int carry = 0;
#pragma unroll
        for (int k = 0; k < SM::NSR; ++k) {
            if (64 * k >= hi_slot) break;
            const int s = lane + 64 * k;
            const int src = (s / BPW) * 4;   // word s / BPW < 64
            const uint64_t w = ((uint64_t)(uint32_t)__builtin_amdgcn_ds_bpermute(src, mhi) << 32) |
                               (uint32_t)__builtin_amdgcn_ds_bpermute(src, mlo);
            const bool mine = s >= lo_slot && s < hi_slot;
            const uint32_t mk = mine ? (uint32_t)(w >> ((s % BPW) * Sh::RC)) & Sh::RCMASK : 0u;
            const int pc = __popc(mk);
            const int incl = wave_scan_dpp(pc);
            sm.put(s, mk, carry + incl - pc);
            carry += __builtin_amdgcn_readlane(incl, 63);
        }
        wave_sync();
        // B. lane = block row: its set bits in turn, every gather issued
        // before the first product; lanes out of bits gather nothing (an out
        // of range offset reads 0) and read the zero in LDS. The slots of a
        // round share one register of block columns (k / R).
        const char *__restrict__ bb = reinterpret_cast<const char *>(sm.w.buf);
        const uint32_t zbyte = (uint32_t)(reinterpret_cast<const char *>(sm.w.zero) - bb);
        const int hi_row = hi_slot * R;
        // G rounds' gathers are issued before the first of their sums: two;
        // four for FP32 with 4-column blocks (half the registers per
        // gather); one for FP64 with one row per block, whose registers
        // would otherwise cost more residency than the overlap gains. With
        // several rounds a round takes at most SC of its block rows' bits
        // (fewer registers); the rare block rows with more take their
        // remaining bits afterwards, in the same order, so the sums are the
        // same.
        constexpr int G = (sizeof(T) == 8 && R == 1) ? 1 : (sizeof(T) == 4 && C == 4) ? 4 : 2;
        constexpr int SC = (G > 1 && C > 4) ? 4 : C;
        double acc[SM::NBR];
#pragma unroll
        for (int k0 = 0; k0 < SM::NBR; k0 += G) {
            if (64 * k0 >= hi_row) break;
            T xg[G][SC], v[G][SC];
            int n[G];             // steps taken per round (uniform)
            uint32_t rest[G];     // bits beyond the first SC
            int colg[G];
            uint32_t voffg[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int k = k0 + g;
                n[g] = 0;
                rest[g] = 0u;
                colg[g] = 0;
                voffg[g] = 0u;
                if (k >= SM::NBR || 64 * k >= hi_row) continue;
                const int br = lane + 64 * k;
                const int s = br / R, rho = br % R;
                const bool ok = s < hi_slot;
                uint32_t mk, first;
                sm.get(ok ? s : 0, mk, first);
                const int col = __builtin_amdgcn_ds_bpermute((s % 64) * 4, in.colr[k / R]);
                mk = ok ? mk : 0u;
                uint32_t rm = (mk >> (rho * C)) & Sh::CMASK;
                const uint32_t voff = (uint32_t)shift + first + (uint32_t)__popc(mk & ((1u << (rho * C)) - 1u));
#pragma unroll
                for (int it = 0; it < SC; ++it) {
                    if (__builtin_amdgcn_ballot_w64(rm != 0u) == 0) break;
                    const bool on = rm != 0u;
                    const int t = __builtin_ctz(rm | (1u << C));
                    xg[g][it] = buf_load<T>(xr, on ? (uint32_t)(col + t) * (uint32_t)sizeof(T) : 0xffffffffu);
                    v[g][it] =
                        *reinterpret_cast<const T *>(bb + (on ? (voff + (uint32_t)it) * (uint32_t)sizeof(T) : zbyte));
                    rm &= rm - 1u;
                    n[g] = it + 1;
                }
                rest[g] = rm;
                colg[g] = col;
                voffg[g] = voff + (uint32_t)SC;
            }
            T sum[G];
#pragma unroll
            for (int g = 0; g < G; ++g) sum[g] = block_row_acc<T, SC>(v[g], xg[g], n[g], T(0));
            if constexpr (SC < C) {
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    uint32_t rm = rest[g];
                    if (__builtin_amdgcn_ballot_w64(rm != 0u) == 0) continue;
                    T x2[C - SC], v2[C - SC];
                    int n2 = 0;
#pragma unroll
                    for (int it = 0; it < C - SC; ++it) {
                        if (__builtin_amdgcn_ballot_w64(rm != 0u) == 0) break;
                        const bool on = rm != 0u;
                        const int t = __builtin_ctz(rm | (1u << C));
                        x2[it] = buf_load<T>(xr, on ? (uint32_t)(colg[g] + t) * (uint32_t)sizeof(T) : 0xffffffffu);
                        v2[it] = *reinterpret_cast<const T *>(
                            bb + (on ? (voffg[g] + (uint32_t)it) * (uint32_t)sizeof(T) : zbyte));
                        rm &= rm - 1u;
                        n2 = it + 1;
                    }
                    sum[g] = block_row_acc<T, C - SC>(v2, x2, n2, sum[g]);
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g)
                if (k0 + g < SM::NBR) acc[k0 + g] = (double)sum[g];
        }
        wave_sync();  // all values are read before the partials overwrite them
        double *__restrict__ part = reinterpret_cast<double *>(sm.w.buf);
#pragma unroll
        for (int k = 0; k < SM::NBR; ++k) {
            if (64 * k >= hi_row) break;
            const int br = lane + 64 * k;
            if (br < hi_row) part[br] = acc[k];   // entry s R + rho
        }
    }
    wave_sync();
    tile_sums<Sh, T, false, 1>(a, d, lo_slot, w0, sm.w.brow, reinterpret_cast<const double *>(sm.w.buf));
}

// One group of block-row rounds: per round, the lane's gathers, its steps,
// its bits, its block column and its first value.
template <class T, int NG_, int SC>
struct BrowGroup {
    static constexpr int NG = NG_;
    T xg[NG][SC];
    int n[NG];             // steps taken per round (uniform)
    uint32_t cnt[NG];      // the bits of the lane's block row
    uint32_t rest[NG];     // bits beyond the first SC
    int colg[NG];
    uint32_t voffg[NG];
};

// Block-row lanes with the first group's gathers ahead of the wait for the
// values (FP64): the arithmetic and its order are brow_run's; pass A's
// results stay in registers for the first group, and the slot table is
// written to LDS after the wait for the groups that follow.
template <class Sh, class T, int KQ>
__device__ void brow_run_early(const SpmvArgs &a, const TileDesc &d, TileIn<Sh, T, KQ, Sh::BPW> &in,
                               __amdgpu_buffer_rsrc_t xr, BrowSmem<Sh, T, KQ> &sm) {
    using SM = BrowSmem<Sh, T, KQ>;
    constexpr int E = SM::W::E;
    constexpr int R = Sh::R, C = Sh::C, BPW = Sh::BPW;
    const int lane = threadIdx.x & 63;
    const T *__restrict__ vals = static_cast<const T *>(a.vals);
    const int b0 = d.b0, b1 = d.b1, nv = d.nv;
    const int64_t abase = d.vbase & ~(int64_t)(E - 1);
    const int shift = (int)(d.vbase - abase);
    const int nq = (shift + nv + E - 1) / E;
    const int q_tail = (abase + (int64_t)nq * E > a.nnz) ? nq - 1 : nq;
    const int w0 = b0 / BPW;
    const int lo_slot = b0 - w0 * BPW;
    const int hi_slot = lo_slot + (b1 - b0);   // the tile's blocks are slots [lo_slot, hi_slot)
    sm.w.brow[lane] = in.br[0] - b0;
    sm.w.brow[lane + 64] = in.br[1] - b0;
    if (lane < 2) sm.w.zero[lane] = 0.0;
    const char *__restrict__ bb = reinterpret_cast<const char *>(sm.w.buf);
    const uint32_t zbyte = (uint32_t)(reinterpret_cast<const char *>(sm.w.zero) - bb);
    const int hi_row = hi_slot * R;
    static_assert(sizeof(T) == 8, "FP64 tiles");
    // brow_run's groups for FP64: G rounds' gathers are issued before the
    // first of their sums (one round with one row per block, else two), and
    // with two rounds a round takes at most SC of its block rows' bits; the
    // rare block rows with more take the rest afterwards, in the same order.
    // The first group, issued while the values stream in, takes up to four
    // rounds with several rows per block and two with one (of up to C bits
    // each): on the 3-D stencil the registers the kernels already hold fit
    // them (2, 3, 6 and 8 rounds were no faster for the former, 1 and 3 for
    // the latter).
    constexpr int G = R == 1 ? 1 : 2;
    constexpr int SC = (G > 1 && C > 4) ? 4 : C;
    constexpr int G0W = R == 1 ? 2 : 4;
    constexpr int G0 = G0W < SM::NBR ? G0W : SM::NBR;
    // pass A's results in registers: round r holds slots 64 r .. 64 r + 63
    uint32_t amk[SM::NSR], afirst[SM::NSR];
    // Issues the gathers of the rounds k0 .. k0 + NG - 1: lane = block row, its
    // set bits in turn; lanes out of bits gather nothing (an out of range
    // offset reads 0). The slots of a round share one register of block
    // columns (k / R), and one of pass A's rounds. The first group takes its
    // slots from pass A's registers (REGS), the others from LDS.
    auto gathers = [&](const int k0, auto &q, const bool REGS) {
        constexpr int NG = std::remove_reference_t<decltype(q)>::NG;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            const int k = k0 + g;
            q.n[g] = 0;
            q.cnt[g] = 0u;
            q.rest[g] = 0u;
            q.colg[g] = 0;
            q.voffg[g] = 0u;
            if (k >= SM::NBR || 64 * k >= hi_row) continue;
            const int br = lane + 64 * k;
            const int s = br / R, rho = br % R;
            const bool ok = s < hi_slot;
            uint32_t mk, first;
            if (REGS) {
                mk = (uint32_t)__builtin_amdgcn_ds_bpermute((s % 64) * 4, (int)amk[k / R]);
                first = (uint32_t)__builtin_amdgcn_ds_bpermute((s % 64) * 4, (int)afirst[k / R]);
            } else {
                sm.get(ok ? s : 0, mk, first);
            }
            const int col = __builtin_amdgcn_ds_bpermute((s % 64) * 4, in.colr[k / R]);
            mk = ok ? mk : 0u;
            uint32_t rm = (mk >> (rho * C)) & Sh::CMASK;
            const uint32_t voff = (uint32_t)shift + first + (uint32_t)__popc(mk & ((1u << (rho * C)) - 1u));
            q.cnt[g] = (uint32_t)__popc(rm);
#pragma unroll
            for (int it = 0; it < SC; ++it) {
                if (__builtin_amdgcn_ballot_w64(rm != 0u) == 0) break;
                const bool on = rm != 0u;
                const int t = __builtin_ctz(rm | (1u << C));
                q.xg[g][it] = buf_load<T>(xr, on ? (uint32_t)(col + t) * (uint32_t)sizeof(T) : 0xffffffffu);
                rm &= rm - 1u;
                q.n[g] = it + 1;
            }
            q.rest[g] = rm;
            q.colg[g] = col;
            q.voffg[g] = voff;
        }
    };
    // The values of the rounds k0 .. k0 + NG - 1 (LDS; the zero for lanes out
    // of bits) and their sums in bit order; block rows with more than SC bits
    // then take the rest.
    auto sums = [&](const int k0, auto &q, double (&acc)[SM::NBR]) {
        constexpr int NG = std::remove_reference_t<decltype(q)>::NG;
        T sum[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            T v[SC];
#pragma unroll
            for (int it = 0; it < SC; ++it) {
                if (it >= q.n[g]) break;
                v[it] = *reinterpret_cast<const T *>(
                    bb + ((uint32_t)it < q.cnt[g] ? (q.voffg[g] + (uint32_t)it) * (uint32_t)sizeof(T) : zbyte));
            }
            sum[g] = block_row_acc<T, SC>(v, q.xg[g], q.n[g], T(0));
        }
        if constexpr (SC < C) {
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                uint32_t rm = q.rest[g];
                if (__builtin_amdgcn_ballot_w64(rm != 0u) == 0) continue;
                T x2[C - SC], v2[C - SC];
                int n2 = 0;
                const uint32_t voff2 = q.voffg[g] + (uint32_t)SC;
#pragma unroll
                for (int it = 0; it < C - SC; ++it) {
                    if (__builtin_amdgcn_ballot_w64(rm != 0u) == 0) break;
                    const bool on = rm != 0u;
                    const int t = __builtin_ctz(rm | (1u << C));
                    x2[it] = buf_load<T>(xr, on ? (uint32_t)(q.colg[g] + t) * (uint32_t)sizeof(T) : 0xffffffffu);
                    v2[it] = *reinterpret_cast<const T *>(
                        bb + (on ? (voff2 + (uint32_t)it) * (uint32_t)sizeof(T) : zbyte));
                    rm &= rm - 1u;
                    n2 = it + 1;
                }
                sum[g] = block_row_acc<T, C - SC>(v2, x2, n2, sum[g]);
            }
        }
#pragma unroll
        for (int g = 0; g < NG; ++g)
            if (k0 + g < SM::NBR) acc[k0 + g] = (double)sum[g];
    };
    // A. lane = slot: its mask bits (from the lane holding its word) and its
    // first value (a prefix over the slots' value counts), kept in registers.
    // Pass A needs only the masks, and the first group's gathers only its
    // results and the block columns, so both run before the wait for the
    // values and the gathers' latency runs under the value stream's. (An LDS
    // access before the wait would wait for the values too: the compiler
    // cannot tell the value loads' LDS destination from the slot table, which
    // is written after.)
    BrowGroup<T, G0, SC> q0;
    if (b1 > b0) {
        const int mlo = (int)(uint32_t)in.m, mhi = (int)(uint32_t)(in.m >> 32);
        int carry = 0;
#pragma unroll
        for (int k = 0; k < SM::NSR; ++k) {
            amk[k] = 0u;
            afirst[k] = 0u;
            if (64 * k >= hi_slot) continue;
            const int s = lane + 64 * k;
            const int src = (s / BPW) * 4;   // word s / BPW < 64
            const uint64_t w = ((uint64_t)(uint32_t)__builtin_amdgcn_ds_bpermute(src, mhi) << 32) |
                               (uint32_t)__builtin_amdgcn_ds_bpermute(src, mlo);
            const bool mine = s >= lo_slot && s < hi_slot;
            const uint32_t mk = mine ? (uint32_t)(w >> ((s % BPW) * Sh::RC)) & Sh::RCMASK : 0u;
            const int pc = __popc(mk);
            const int incl = wave_scan_dpp(pc);
            amk[k] = mk;
            afirst[k] = (uint32_t)(carry + incl - pc);
            carry += __builtin_amdgcn_readlane(incl, 63);
        }
        gathers(0, q0, true);
    }
    wait_vm_all();   // the values have landed in LDS; the chunk past nnz is filled value by value
    if (q_tail < nq && lane < E) {
        const int64_t g = abase + (int64_t)q_tail * E + lane;
        if (g < a.nnz) sm.w.buf[q_tail * E + lane] = vals[g];
    }
    if (b1 > b0 && SM::NBR > G0) {   // the slot table, for the groups after the first
#pragma unroll
        for (int k = 0; k < SM::NSR; ++k) {
            if (64 * k >= hi_slot) break;
            sm.put(lane + 64 * k, amk[k], afirst[k]);
        }
    }
    wave_sync();
    if (b1 > b0) {
        // B. lane = block row: G rounds at a time, every gather of a group
        // issued before its first product
        double acc[SM::NBR];
        sums(0, q0, acc);
#pragma unroll
        for (int k0 = G0; k0 < SM::NBR; k0 += G) {
            if (64 * k0 >= hi_row) break;
            BrowGroup<T, G, SC> q;
            gathers(k0, q, false);
            sums(k0, q, acc);
        }
        wave_sync();  // all values are read before the partials overwrite them
        double *__restrict__ part = reinterpret_cast<double *>(sm.w.buf);
#pragma unroll
        for (int k = 0; k < SM::NBR; ++k) {
            if (64 * k >= hi_row) break;
            const int br = lane + 64 * k;
            if (br < hi_row) part[br] = acc[k];   // entry s R + rho
        }
    }
    wave_sync();
    tile_sums<Sh, T, false, 1>(a, d, lo_slot, w0, sm.w.brow, reinterpret_cast<const double *>(sm.w.buf));
}

template <class Sh, class T, int KQ>
__device__ __forceinline__ void brow_tile(const SpmvArgs &a, const TileDesc &d, __amdgpu_buffer_rsrc_t xr,
                                          BrowSmem<Sh, T, KQ> &sm) {
    TileIn<Sh, T, KQ, Sh::BPW> in;
    tile_issue<Sh, T, KQ>(a, d, in, sm.w.buf);
    // FP64 gathers before the wait; FP32 after it (measured faster for each)
    if constexpr (sizeof(T) == 8) brow_run_early<Sh, T, KQ>(a, d, in, xr, sm);
    else brow_run<Sh, T, KQ>(a, d, in, xr, sm);
}

// ---------------------------------------------------------------------------
// Value lanes (mode 4, beta(1,8)): the tiles of mode 3, with one lane per
// stored value. With one row per block, the values of a row are contiguous
// in the packed array, so the product pass needs only each value's column:
//   A. lane = slot: its mask byte, its first value (a prefix over the
//      slots' value counts), then its columns, written to LDS at the ranks
//      of its values (as many steps as the fullest block has values);
//   B. lane = value: column and value from LDS, one x gather, the product
//      replacing the value in LDS (FP32: the product rounded to float);
//   C. L lanes per row add the row's contiguous products in double and
//      combine their sums with shuffles.
// Every lane of the gather pass holds a stored value, and the lanes of one
// block read neighbouring x entries in the same instruction.
template <class Sh, class T, int KQ>
struct VlaneSmem {
    static_assert(Sh::R == 1, "value lanes need one row per block");
    using B = BrowSmem<Sh, T, KQ>;
    static constexpr int NS = B::NS, NSR = B::NSR, VCAP = B::VCAP, NBX = B::NBX;
    static constexpr int NVR = (VCAP + 63) / 64;   // 64-lane rounds over a tile's values
    typename B::W w;        // values, then products; interval pointers; zero
    static_assert(VCAP < 65536, "first values fit 16 bits");
    uint16_t first[NS];     // first value of each slot (tile-relative)
    int col[VCAP];          // column of each value
};

template <class Sh, class T, int KQ>
__device__ void vlane_run(const SpmvArgs &a, const TileDesc &d, TileIn<Sh, T, KQ, Sh::BPW> &in,
                          __amdgpu_buffer_rsrc_t xr, VlaneSmem<Sh, T, KQ> &sm) {
    using SM = VlaneSmem<Sh, T, KQ>;
    constexpr int E = SM::B::W::E;
    constexpr int BPW = Sh::BPW;
    const int lane = threadIdx.x & 63;
    const T *__restrict__ vals = static_cast<const T *>(a.vals);
    const int b0 = d.b0, b1 = d.b1, nv = d.nv;
    const int64_t abase = d.vbase & ~(int64_t)(E - 1);
    const int shift = (int)(d.vbase - abase);
    const int nq = (shift + nv + E - 1) / E;
    const int q_tail = (abase + (int64_t)nq * E > a.nnz) ? nq - 1 : nq;
    const int w0 = b0 / BPW;
    const int lo_slot = b0 - w0 * BPW;
    const int nb = b1 - b0;
    const int hi_slot = lo_slot + nb;
    sm.w.brow[lane] = in.br[0] - b0;
    sm.w.brow[lane + 64] = in.br[1] - b0;
    wait_vm_all();   // the values have landed in LDS; the chunk past nnz is filled value by value
    if (q_tail < nq && lane < E) {
        const int64_t g = abase + (int64_t)q_tail * E + lane;
        if (g < a.nnz) sm.w.buf[q_tail * E + lane] = vals[g];
    }
    if (nb > 0) {
        // A. lane = slot: mask byte, first value, then its columns by rank
        const int mlo = (int)(uint32_t)in.m, mhi = (int)(uint32_t)(in.m >> 32);
        int carry = 0;
#pragma unroll
        for (int k = 0; k < SM::NSR; ++k) {
            if (64 * k >= hi_slot) break;
            const int s = lane + 64 * k;
            const int src = (s / BPW) * 4;
            const uint64_t w = ((uint64_t)(uint32_t)__builtin_amdgcn_ds_bpermute(src, mhi) << 32) |
                               (uint32_t)__builtin_amdgcn_ds_bpermute(src, mlo);
            const bool mine = s >= lo_slot && s < hi_slot;
            uint32_t rm = mine ? (uint32_t)(w >> ((s % BPW) * Sh::RC)) & Sh::RCMASK : 0u;
            const int pc = __popc(rm);
            const int incl = wave_scan_dpp(pc);
            const int first = carry + incl - pc;
            sm.first[s] = (uint16_t)first;
            carry += __builtin_amdgcn_readlane(incl, 63);
            const int col0 = in.colr[k];
#pragma unroll
            for (int it = 0; it < Sh::C; ++it) {
                if (__builtin_amdgcn_ballot_w64(rm != 0u) == 0) break;
                if (rm != 0u) sm.col[first + it] = col0 + __builtin_ctz(rm);
                rm &= rm - 1u;
            }
        }
        wave_sync();
        // B. lane = value, eight rounds of gathers in flight at a time
        T *__restrict__ vb = sm.w.buf + shift;
        constexpr int U = 8;
#pragma unroll
        for (int q0 = 0; q0 < SM::NVR; q0 += U) {
            if (64 * q0 >= nv) break;
            T xg[U], vv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int v = lane + 64 * (q0 + u);
                const bool on = q0 + u < SM::NVR && v < nv;
                const int c = sm.col[on ? v : 0];
                xg[u] = buf_load<T>(xr, on ? (uint32_t)c * (uint32_t)sizeof(T) : 0xffffffffu);
                vv[u] = on ? vb[v] : T(0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int v = lane + 64 * (q0 + u);
                if (q0 + u < SM::NVR && v < nv) vb[v] = vv[u] * xg[u];
            }
        }
        wave_sync();
    }
    // C. row sums: L lanes per row (the largest L with rows * L <= 64; with
    // more than 64 rows a lane takes rows lane and lane + 64)
    const int nI = d.i1 - d.i0;
    const int lg = nI > 64 ? 0 : nI > 1 ? __builtin_clz((unsigned)(nI - 1)) - 26 : 6;
    const int L = 1 << lg;
    const int l = lane & (L - 1);
    const T *__restrict__ pb = sm.w.buf + shift;
    for (int round = 0; round < 2; ++round) {
        if (round == 1 && nI <= 64) break;
        const int li = (lane >> lg) + 64 * round;
        double acc = 0.0;
        bool stored = false;
        if (li < nI) {
            const int bs = sm.w.brow[li], be = sm.w.brow[li + 1];   // tile-relative blocks
            stored = be > bs;   // every block holds at least one value
            const int vs = bs < nb ? sm.first[bs + lo_slot] : nv;
            const int ve = be < nb ? sm.first[be + lo_slot] : nv;
            double a0 = 0.0, a1 = 0.0;
            int v = vs + l;
            for (; v + L < ve; v += 2 * L) {
                a0 += (double)pb[v];
                a1 += (double)pb[v + L];
            }
            if (v < ve) a0 += (double)pb[v];
            acc = a0 + a1;
        }
        acc = group_sum(acc, lg);
        if (li < nI && l == 0) {
            const int64_t row = (int64_t)d.i0 + li;
            if (row < a.n_rows) {
                T *__restrict__ y = static_cast<T *>(a.y);
                if (a.accumulate) {
                    if (stored) y[row] = (T)(acc + (double)y[row]);
                } else {
                    y[row] = (T)acc;
                }
            }
        }
    }
}

template <class Sh, class T, int KQ>
__device__ __forceinline__ void vlane_tile(const SpmvArgs &a, const TileDesc &d, __amdgpu_buffer_rsrc_t xr,
                                           VlaneSmem<Sh, T, KQ> &sm) {
    TileIn<Sh, T, KQ, Sh::BPW> in;
    tile_issue<Sh, T, KQ>(a, d, in, sm.w.buf);
    vlane_run<Sh, T, KQ>(a, d, in, xr, sm);
}

// The KQ 16-byte chunks of a wavefront's value range, lane l taking bytes
// 16 l of each 1 KB, straight into LDS (chunk k at s_vals + 64 k E).
template <class T, int KQ>
__device__ __forceinline__ void values_to_lds(__amdgpu_buffer_rsrc_t vr, T *s_vals) {
    constexpr int E = 16 / sizeof(T);
    const int lane = lane_id();
#pragma unroll
    for (int k = 0; k < KQ; ++k)
        chunk_to_lds(vr, s_vals + 64 * k * E, (uint32_t)(lane * 16), 1024 * k);
}

using V4u = __attribute__((ext_vector_type(4))) unsigned int;

// The streams of a tile as tile_issue issues them; with TO_LDS = false the
// packed values go to registers (v[k]: chunk k, lane l's 16 bytes at
// 1024 k + 16 l), so that while an earlier tile is worked on they hold no
// LDS. NCR + 3 + KQ loads, all unguarded buffer loads.
template <class Sh, class T, int KQ, bool TO_LDS>
__device__ __forceinline__ void tile_issue_regs(const SpmvArgs &a, const TileDesc &d, TileIn<Sh, T, KQ> &in,
                                                V4u (&v)[KQ], T *s_vals) {
    using SM = WaveSmem<Sh, T, KQ>;
    constexpr int E = SM::E;
    const int lane = lane_id();
    const T *__restrict__ vals = static_cast<const T *>(a.vals);
    const int b0 = d.b0, b1 = d.b1, nv = d.nv, nI = d.i1 - d.i0;
    const int64_t abase = d.vbase & ~(int64_t)(E - 1);
    const int shift = (int)(d.vbase - abase);
    const int nq = (shift + nv + E - 1) / E;
    const int q_tail = (abase + (int64_t)nq * E > a.nnz) ? nq - 1 : nq;
    const int w0 = b0 / Sh::BPW;
    const int nw = (b1 > b0) ? ((b1 - 1) / Sh::BPW - w0 + 1) : 0;
    const int cs0 = w0 * Sh::BPW;
    const int ncs = (int)(min<int64_t>((int64_t)(w0 + nw) * Sh::BPW, a.n_blocks) - cs0);
    const auto cr = rsrc(a.bcol + cs0, (uint32_t)ncs * 4u);
#pragma unroll
    for (int k = 0; k < SM::NCR; ++k)
        in.colr[k] = __builtin_amdgcn_raw_buffer_load_b32(cr, (uint32_t)(lane * 4), 256 * k, kNT);
    const auto brr = rsrc(a.brow + d.i0, (uint32_t)(nI + 1) * 4u);
    in.br[0] = __builtin_amdgcn_raw_buffer_load_b32(brr, (uint32_t)(lane * 4), 0, 0);
    in.br[1] = __builtin_amdgcn_raw_buffer_load_b32(brr, (uint32_t)(lane * 4), 256, 0);
    const auto mr = rsrc(a.mw + w0, (uint32_t)nw * 8u);
    in.m = __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(mr, (uint32_t)(lane * 8), 0, kNT));
    const auto vr = rsrc(vals + abase, (uint32_t)q_tail * 16u);
    if constexpr (TO_LDS) {
        values_to_lds<T, KQ>(vr, s_vals);
    } else {
#pragma unroll
        for (int k = 0; k < KQ; ++k)
            v[k] = __builtin_amdgcn_raw_buffer_load_b128(vr, (uint32_t)(lane * 16), 1024 * k, kNT);
    }
}

// Two consecutive tiles on one wavefront: the first tile's values go straight
// to LDS, the second tile's to registers, and both tiles' streams are in
// flight together; the first tile is worked on as soon as its own loads have
// landed, then the second tile's values are written to the same LDS buffer.
// A wavefront thus keeps two tiles' bytes in flight for one tile's LDS.
template <class Sh, class T, int KQ>
__device__ void wave_tile_pair(const SpmvArgs &a, const TileDesc &d0, const TileDesc &d1,
                               __amdgpu_buffer_rsrc_t xr, WaveSmem<Sh, T, KQ> &sm) {
    using SM = WaveSmem<Sh, T, KQ>;
    constexpr int E = SM::E;
    constexpr int PEND = SM::NCR + 3 + KQ;     // loads of tile_issue_regs
    TileIn<Sh, T, KQ> in0, in1;
    V4u v1[KQ];
    tile_issue_regs<Sh, T, KQ, true>(a, d0, in0, v1, sm.buf);
    tile_issue_regs<Sh, T, KQ, false>(a, d1, in1, v1, sm.buf);
    tile_run<Sh, T, KQ, PEND>(a, d0, in0, xr, sm);
    wave_sync();  // the first tile's LDS reads are done before its buffer is refilled
    const int lane = lane_id();
#pragma unroll
    for (int k = 0; k < KQ; ++k) *reinterpret_cast<V4u *>(&sm.buf[(lane + 64 * k) * E]) = v1[k];
    tile_run<Sh, T, KQ, -1>(a, d1, in1, xr, sm);
}

// One interval longer than a wavefront tile, run by one wavefront: each lane
// keeps the running sum of its block row over all the interval's words.
template <class Sh, class T>
__device__ void wave_long(const SpmvArgs &a, int I, int b0, int b1, int64_t vbase) {
    const int lane = threadIdx.x & 63;
    const T *__restrict__ vals = static_cast<const T *>(a.vals);
    const T *__restrict__ x = static_cast<const T *>(a.x);
    const int slot = lane / Sh::RC;
    const int kcol = (lane % Sh::RC) % Sh::C;
    const int w0 = b0 / Sh::BPW;
    const int nwt = (b1 - 1) / Sh::BPW - w0 + 1;
    double acc0 = 0.0, acc1 = 0.0;
    int n_here = 0;  // stored entries this lane saw
    int64_t vrun = vbase;
    for (int k = 0; k < nwt; k += 64) {
        const int nw = min(64, nwt - k);
        const uint64_t wm = tile_word<Sh>(a.mw, w0 + k, nw, b0, b1, lane);
        const int cnt = __popcll(wm);
        const int incl = wave_incl_scan(cnt);
        const int excl = incl - cnt;
        for (int i = 0; i < nw; i += kUnroll) {
            uint64_t M[kUnroll];
            int off[kUnroll];
            unsigned rk[kUnroll];
            bool act[kUnroll];
            int col[kUnroll];
            T v[kUnroll], xv[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const bool in = (i + u) < nw;
                M[u] = in ? readlane64(wm, i + u) : 0ull;
                off[u] = in ? __builtin_amdgcn_readlane(excl, i + u) : 0;
                act[u] = (M[u] >> lane) & 1ull;
                rk[u] = lane_rank(M[u]);
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (act[u]) {
                    col[u] = ldg_nt(a.bcol + (int64_t)(w0 + k + i + u) * Sh::BPW + slot) + kcol;
                    v[u] = ldg_nt(vals + vrun + off[u] + rk[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                if (act[u]) xv[u] = x[col[u]];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (act[u]) {
                    ++n_here;
                    if (u & 1) acc1 = __builtin_fma((double)v[u], (double)xv[u], acc1);
                    else acc0 = __builtin_fma((double)v[u], (double)xv[u], acc0);
                }
            }
        }
        vrun += __builtin_amdgcn_readlane(incl, nw - 1);
    }
    double acc = acc0 + acc1;
    // sums over lanes of the same block row: xor over column bits, then slot bits
#pragma unroll
    for (int m = 1; m < Sh::C; m <<= 1) {
        acc += __shfl_xor(acc, m, 64);
        n_here += __shfl_xor(n_here, m, 64);
    }
#pragma unroll
    for (int m = Sh::RC; m < 64; m <<= 1) {
        acc += __shfl_xor(acc, m, 64);
        n_here += __shfl_xor(n_here, m, 64);
    }
    if (lane < Sh::RC && (lane % Sh::C) == 0) {
        const int rho = lane / Sh::C;
        const int64_t row = (int64_t)I * Sh::R + rho;
        if (row < a.n_rows) {
            T *__restrict__ y = static_cast<T *>(a.y);
            if (a.accumulate) {
                if (n_here > 0) y[row] = (T)(acc + (double)y[row]);
            } else {
                y[row] = (T)acc;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// One interval with more blocks than a tile holds.
template <class Sh, class T>
__device__ void tile_long(const SpmvArgs &a, int I, int b0, int b1, int64_t vbase, double *s_red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const T *__restrict__ vals = static_cast<const T *>(a.vals);
    const T *__restrict__ x = static_cast<const T *>(a.x);
    const int slot = lane / Sh::RC;
    const int kcol = (lane % Sh::RC) % Sh::C;
    const int w0 = b0 / Sh::BPW;
    const int nwt = (b1 - 1) / Sh::BPW - w0 + 1;
    double acc0 = 0.0, acc1 = 0.0;
    int64_t vrun = vbase;
    for (int k = 0; k < nwt; k += 64) {
        const int nw = min(64, nwt - k);
        const uint64_t wm = tile_word<Sh>(a.mw, w0 + k, nw, b0, b1, lane);
        const int cnt = __popcll(wm);
        const int incl = wave_incl_scan(cnt);
        const int excl = incl - cnt;
        for (int i = wid; i < nw; i += kWaves * kUnroll) {
            uint64_t M[kUnroll];
            int off[kUnroll];
            unsigned rk[kUnroll];
            bool act[kUnroll];
            int col[kUnroll];
            T v[kUnroll], xv[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int ii = i + u * kWaves;
                const bool in = ii < nw;
                M[u] = in ? readlane64(wm, ii) : 0ull;
                off[u] = in ? __builtin_amdgcn_readlane(excl, ii) : 0;
                act[u] = (M[u] >> lane) & 1ull;
                rk[u] = lane_rank(M[u]);
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (act[u]) {
                    col[u] = ldg_nt(a.bcol + (int64_t)(w0 + k + i + u * kWaves) * Sh::BPW + slot) + kcol;
                    v[u] = ldg_nt(vals + vrun + off[u] + rk[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                if (act[u]) xv[u] = x[col[u]];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (act[u]) {
                    if (u & 1) acc1 = __builtin_fma((double)v[u], (double)xv[u], acc1);
                    else acc0 = __builtin_fma((double)v[u], (double)xv[u], acc0);
                }
            }
        }
        vrun += __builtin_amdgcn_readlane(incl, nw - 1);
    }
    double acc = acc0 + acc1;
    // lanes of one block row: same (lane % RC) / C; add over column and slot bits
#pragma unroll
    for (int m = 1; m < Sh::C; m <<= 1) acc += __shfl_xor(acc, m, 64);
#pragma unroll
    for (int m = Sh::RC; m < 64; m <<= 1) acc += __shfl_xor(acc, m, 64);
    if (lane < Sh::RC && (lane % Sh::C) == 0) s_red[wid * Sh::R + lane / Sh::C] = acc;
    __syncthreads();
    if ((int)threadIdx.x < Sh::R) {
        const int rho = threadIdx.x;
        double s = 0.0;
        for (int w = 0; w < kWaves; ++w) s += s_red[w * Sh::R + rho];
        const int64_t row = (int64_t)I * Sh::R + rho;
        if (row < a.n_rows) {
            T *__restrict__ y = static_cast<T *>(a.y);
            if (a.accumulate) s += (double)y[row];
            y[row] = (T)s;
        }
    }
}

// Mode 1: one workgroup per tile (lane = mask bit throughout).
template <int R, int C, class T, int TB>
__global__ __launch_bounds__(kThreads) void k_spmv_wg(SpmvArgs a) {
    using Sh = Shape<R, C>;
    static_assert(TB / 64 + 1 <= 64, "a tile must fit 64 mask words");
    __shared__ double s_red[kWaves * 8];
    __shared__ uint64_t s_wm[TB / 64 + 2];
    __shared__ int s_off[TB / 64 + 2];
    __shared__ T s_prod[TB];
    int t = blockIdx.x;
    if (a.xcd_remap) t = (int)(blockIdx.x & 7u) * a.tiles_per_xcd + (int)(blockIdx.x >> 3);
    if (t >= a.n_tiles) return;
    const TileDesc d = a.tiles[t];
    const int b0 = a.brow[d.i0], b1 = a.brow[d.i1];
    if (b1 - b0 > TB / Sh::RC) tile_long<Sh, T>(a, d.i0, b0, b1, d.vbase, s_red);
    else tile_short<Sh, T, TB>(a, d.i0, d.i1, b0, b1, d.vbase, s_wm, s_off, s_prod);
}

// Mode 0: one wavefront per tile, four independent tiles per workgroup.
template <int R, int C, class T, int KQ>
__global__ __launch_bounds__(kThreads) void k_spmv_wave(SpmvArgs a) {
    using Sh = Shape<R, C>;
    using SM = WaveSmem<Sh, T, KQ>;
    __shared__ SM sm[kWaves];
    int g = blockIdx.x;
    if (a.xcd_remap) g = (int)(blockIdx.x & 7u) * a.tiles_per_xcd + (int)(blockIdx.x >> 3);
    // the wavefront index is uniform; say so, so that everything derived from
    // it (tile, block range, mask words) lives in scalar registers
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = g * kWaves + wid;
    if (t >= a.n_tiles) return;
    const TileDesc d = a.tiles[t];
    if (d.b1 - d.b0 > SM::NB) {
        wave_long<Sh, T>(a, d.i0, d.b0, d.b1, d.vbase);
    } else {
        const auto xr = rsrc(a.x, (uint32_t)(a.n_cols * (int64_t)sizeof(T)));
        wave_tile<Sh, T, KQ>(a, d, xr, sm[wid]);
    }
}

// Mode 3: one block-row-lane tile per wavefront; an interval beyond a
// tile's values or blocks takes mode 0's long path.
template <int R, int C, class T, int KQ>
__global__ __launch_bounds__(kThreads) void k_spmv_brow(SpmvArgs a) {
    using Sh = Shape<R, C>;
    using SM = BrowSmem<Sh, T, KQ>;
    __shared__ SM sm[kWaves];
    int g = blockIdx.x;
    if (a.xcd_remap) g = (int)(blockIdx.x & 7u) * a.tiles_per_xcd + (int)(blockIdx.x >> 3);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = g * kWaves + wid;
    if (t >= a.n_tiles) return;
    const TileDesc d = a.tiles[t];
    if (d.b1 - d.b0 > SM::NBX || d.nv > SM::VCAP) {
        wave_long<Sh, T>(a, d.i0, d.b0, d.b1, d.vbase);
    } else {
        const auto xr = rsrc(a.x, (uint32_t)(a.n_cols * (int64_t)sizeof(T)));
        brow_tile<Sh, T, KQ>(a, d, xr, sm[wid]);
    }
}

// Mode 4: one value-lane tile per wavefront (beta(1,8)); an interval beyond
// a tile's values or blocks takes mode 0's long path.
template <class T, int KQ>
__global__ __launch_bounds__(kThreads) void k_spmv_vlane(SpmvArgs a) {
    using Sh = Shape<1, 8>;
    using SM = VlaneSmem<Sh, T, KQ>;
    __shared__ SM sm[kWaves];
    int g = blockIdx.x;
    if (a.xcd_remap) g = (int)(blockIdx.x & 7u) * a.tiles_per_xcd + (int)(blockIdx.x >> 3);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = g * kWaves + wid;
    if (t >= a.n_tiles) return;
    const TileDesc d = a.tiles[t];
    if (d.b1 - d.b0 > SM::NBX || d.nv > SM::VCAP) {
        wave_long<Sh, T>(a, d.i0, d.b0, d.b1, d.vbase);
    } else {
        const auto xr = rsrc(a.x, (uint32_t)(a.n_cols * (int64_t)sizeof(T)));
        vlane_tile<Sh, T, KQ>(a, d, xr, sm[wid]);
    }
}

// Mode 0 with two consecutive tiles per wavefront (wave_tiles = 2).
template <int R, int C, class T, int KQ>
__global__ __launch_bounds__(kThreads) void k_spmv_wave2(SpmvArgs a) {
    using Sh = Shape<R, C>;
    using SM = WaveSmem<Sh, T, KQ>;
    __shared__ SM sm[kWaves];
    int g = blockIdx.x;
    if (a.xcd_remap) g = (int)(blockIdx.x & 7u) * a.tiles_per_xcd + (int)(blockIdx.x >> 3);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t0 = 2 * (g * kWaves + wid);
    if (t0 >= a.n_tiles) return;
    const bool has1 = t0 + 1 < a.n_tiles;
    const TileDesc d0 = a.tiles[t0];
    const TileDesc d1 = a.tiles[has1 ? t0 + 1 : t0];
    const auto xr = rsrc(a.x, (uint32_t)(a.n_cols * (int64_t)sizeof(T)));
    const bool long0 = d0.b1 - d0.b0 > SM::NB, long1 = d1.b1 - d1.b0 > SM::NB;
    if (has1 && !long0 && !long1) {
        wave_tile_pair<Sh, T, KQ>(a, d0, d1, xr, sm[wid]);
        return;
    }
    // a long interval on either side: the two tiles one after the other
    if (long0) wave_long<Sh, T>(a, d0.i0, d0.b0, d0.b1, d0.vbase);
    else wave_tile<Sh, T, KQ>(a, d0, xr, sm[wid]);
    if (has1) {
        wave_sync();
        if (long1) wave_long<Sh, T>(a, d1.i0, d1.b0, d1.b1, d1.vbase);
        else wave_tile<Sh, T, KQ>(a, d1, xr, sm[wid]);
    }
}

// ---------------------------------------------------------------------------
// Batched: tiles of many matrices in one launch. A wavefront reads its tile,
// the tile's matrix (TileDesc::reserved) and switches on that matrix's shape;
// tile, matrix and shape are uniform across the wavefront, so the switch is a
// scalar branch. The LDS of a wavefront is the largest of the six layouts.
template <class T, int KQ>
union BatchSmem {
    WaveSmem<Shape<1, 8>, T, KQ> s0;
    WaveSmem<Shape<2, 4>, T, KQ> s1;
    WaveSmem<Shape<2, 8>, T, KQ> s2;
    WaveSmem<Shape<4, 4>, T, KQ> s3;
    WaveSmem<Shape<4, 8>, T, KQ> s4;
    WaveSmem<Shape<8, 4>, T, KQ> s5;
};

// The product arguments of one matrix of a batch.
__device__ __forceinline__ SpmvArgs batch_args(const BatchMat &M, const TileDesc *tiles, int accumulate) {
    SpmvArgs a;
    a.brow = M.brow;
    a.bcol = M.bcol;
    a.mw = M.mw;
    a.vals = M.vals;
    a.x = M.x;
    a.y = M.y;
    a.tiles = tiles;
    a.n_rows = M.n_rows;
    a.nnz = M.nnz;
    a.n_blocks = M.n_blocks;
    a.n_cols = M.n_cols;
    a.n_tiles = 0;
    a.accumulate = accumulate;
    a.xcd_remap = 0;
    a.tiles_per_xcd = 0;
    return a;
}

template <class Sh, class T, int KQ>
__device__ __forceinline__ void batched_tile(const SpmvArgs &a, const TileDesc &d, WaveSmem<Sh, T, KQ> &sm) {
    if (d.b1 - d.b0 > WaveSmem<Sh, T, KQ>::NB) {
        wave_long<Sh, T>(a, d.i0, d.b0, d.b1, d.vbase);
    } else {
        const auto xr = rsrc(a.x, (uint32_t)(a.n_cols * (int64_t)sizeof(T)));
        wave_tile<Sh, T, KQ>(a, d, xr, sm);
    }
}

template <class T, int KQ, bool PERSIST>
__global__ __launch_bounds__(kThreads) void k_spmv_batched(const BatchMat *__restrict__ mats,
                                                           const TileDesc *__restrict__ tiles, int64_t n_tiles,
                                                           int accumulate) {
    __shared__ BatchSmem<T, KQ> sm[kWaves];
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t0 = (int64_t)blockIdx.x * kWaves + wid;
    const int64_t step = PERSIST ? (int64_t)gridDim.x * kWaves : n_tiles;
    for (int64_t t = t0; t < n_tiles; t += step) {
        const TileDesc d = tiles[t];
        const BatchMat &M = mats[d.reserved];
        const SpmvArgs a = batch_args(M, tiles, accumulate);
        wave_sync();  // the previous tile's LDS reads are done before this tile writes
        switch (M.shape) {
        case 0: batched_tile<Shape<1, 8>, T, KQ>(a, d, sm[wid].s0); break;
        case 1: batched_tile<Shape<2, 4>, T, KQ>(a, d, sm[wid].s1); break;
        case 2: batched_tile<Shape<2, 8>, T, KQ>(a, d, sm[wid].s2); break;
        case 3: batched_tile<Shape<4, 4>, T, KQ>(a, d, sm[wid].s3); break;
        case 4: batched_tile<Shape<4, 8>, T, KQ>(a, d, sm[wid].s4); break;
        default: batched_tile<Shape<8, 4>, T, KQ>(a, d, sm[wid].s5); break;
        }
    }
}

// A batch whose matrices all have shape S: no switch, and only that shape's
// LDS layout, so occupancy matches the single-matrix kernel.
// PERSIST = false: one tile per wavefront (the grid covers the list), no loop.
template <int S, class T, int KQ, bool PERSIST>
__global__ __launch_bounds__(kThreads) void k_spmv_batched_fixed(const BatchMat *__restrict__ mats,
                                                                 const TileDesc *__restrict__ tiles, int64_t n_tiles,
                                                                 int accumulate) {
    using Sh = Shape<kShapeR[S], kShapeC[S]>;
    __shared__ WaveSmem<Sh, T, KQ> sm[kWaves];
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t0 = (int64_t)blockIdx.x * kWaves + wid;
    const int64_t step = PERSIST ? (int64_t)gridDim.x * kWaves : n_tiles;
    for (int64_t t = t0; t < n_tiles; t += step) {
        const TileDesc d = tiles[t];
        const SpmvArgs a = batch_args(mats[d.reserved], tiles, accumulate);
        wave_sync();
        batched_tile<Sh, T, KQ>(a, d, sm[wid]);
    }
}

template <int S, class T, bool P>
void launch_batched_fixed_p(int kq, unsigned grid, const BatchMat *d_mats, const TileDesc *d_tiles,
                            int64_t n_tiles, int accumulate, hipStream_t stream) {
    switch (kq) {
    case 2:
        hipLaunchKernelGGL((k_spmv_batched_fixed<S, T, 2, P>), dim3(grid), dim3(kThreads), 0, stream, d_mats,
                           d_tiles, n_tiles, accumulate);
        break;
    case 6:
        hipLaunchKernelGGL((k_spmv_batched_fixed<S, T, 6, P>), dim3(grid), dim3(kThreads), 0, stream, d_mats,
                           d_tiles, n_tiles, accumulate);
        break;
    case 8:
        hipLaunchKernelGGL((k_spmv_batched_fixed<S, T, 8, P>), dim3(grid), dim3(kThreads), 0, stream, d_mats,
                           d_tiles, n_tiles, accumulate);
        break;
    default:
        hipLaunchKernelGGL((k_spmv_batched_fixed<S, T, 4, P>), dim3(grid), dim3(kThreads), 0, stream, d_mats,
                           d_tiles, n_tiles, accumulate);
        break;
    }
}

template <int S, class T>
void launch_batched_fixed(int kq, unsigned grid, bool persist, const BatchMat *d_mats, const TileDesc *d_tiles,
                          int64_t n_tiles, int accumulate, hipStream_t stream) {
    if (persist) launch_batched_fixed_p<S, T, true>(kq, grid, d_mats, d_tiles, n_tiles, accumulate, stream);
    else launch_batched_fixed_p<S, T, false>(kq, grid, d_mats, d_tiles, n_tiles, accumulate, stream);
}

// Mode 0, pipelined: a persistent grid; each wavefront walks the tiles
// t, t + S, t + 2S, ... (S = 4 x grid). The packed values travel from memory
// straight into LDS (buffer loads with the LDS destination), so a tile's
// values can be in flight while the previous tile is computed without
// holding any registers. A wavefront has one value buffer: a tile's values
// leave it for registers (with their x gathers) before the next tile's
// values are requested into it, and the tile's partials go to an area of
// their own. Per tile:
//   wait for everything issued so far (this tile's streams, loaded during
//   the previous tile); read the values and issue the x gathers; issue the
//   next tile's streams (block columns, interval pointers, mask words, the
//   descriptor after it) and its values; compute this tile.
// Vector memory operations complete in issue order, so waiting for the
// gathers does not wait for the next tile's streams.
template <class Sh, class T, int KQ>
struct PipeSmem {
    static constexpr int NBUF = WaveSmem<Sh, T, KQ>::NBUF;
    T buf[NBUF];
    // the partials and the interval pointers follow buf, so that the value
    // reads of the last word's lanes past the tile (at most 63 entries past
    // buf, never used) stay inside this wavefront's own area
    double part[WaveSmem<Sh, T, KQ>::NPART];
    int brow[128];
    double zero[2];   // read by the lanes of clear mask bits
};

template <class Sh, class T, int KQ>
struct TileNext {
    int colr[WaveSmem<Sh, T, KQ>::NCR];
    int br[2];
    uint64_t m;  // lane j: the tile's mask word j (0 past the tile's words)
};


// Lanes 0..7 load the eight dwords of descriptor t.
__device__ __forceinline__ int desc_lane(const SpmvArgs &a, int t) {
    const int lane = threadIdx.x & 63;
    const auto r = rsrc(a.tiles, (uint32_t)a.n_tiles * (uint32_t)sizeof(TileDesc));
    const uint32_t off = lane < 8 ? (uint32_t)t * (uint32_t)sizeof(TileDesc) + 4u * (uint32_t)lane : 0xffffffffu;
    return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}

__device__ __forceinline__ TileDesc desc_from_lanes(int v) {
    TileDesc d;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane(v, 0), hi = (uint32_t)__builtin_amdgcn_readlane(v, 1);
    d.vbase = (int64_t)(((uint64_t)hi << 32) | lo);
    d.i0 = __builtin_amdgcn_readlane(v, 2);
    d.i1 = __builtin_amdgcn_readlane(v, 3);
    d.b0 = __builtin_amdgcn_readlane(v, 4);
    d.b1 = __builtin_amdgcn_readlane(v, 5);
    d.nv = __builtin_amdgcn_readlane(v, 6);
    d.reserved = __builtin_amdgcn_readlane(v, 7);
    return d;
}

// Issues a tile's streams: registers for the small ones, LDS (s_vals) for
// the packed values. All loads are unguarded buffer loads. With on = false
// the same loads are issued with empty ranges (they return zeros and touch no
// memory), so the number of memory operations in flight does not depend on
// a branch and the waits for earlier loads stay exact.
template <class Sh, class T, int KQ>
__device__ __forceinline__ void tile_issue_lds(const SpmvArgs &a, const TileDesc &d, TileNext<Sh, T, KQ> &in,
                                               T *s_vals, bool on) {
    using SM = WaveSmem<Sh, T, KQ>;
    constexpr int E = SM::E;
    const int lane = threadIdx.x & 63;
    const T *__restrict__ vals = static_cast<const T *>(a.vals);
    const int b0 = d.b0, b1 = d.b1, nv = d.nv, nI = d.i1 - d.i0;
    const int64_t abase = d.vbase & ~(int64_t)(E - 1);
    const int shift = (int)(d.vbase - abase);
    const int nq = (shift + nv + E - 1) / E;
    const int q_tail = (abase + (int64_t)nq * E > a.nnz) ? nq - 1 : nq;
    const int w0 = b0 / Sh::BPW;
    const int nw = (b1 > b0) ? ((b1 - 1) / Sh::BPW - w0 + 1) : 0;
    const int cs0 = w0 * Sh::BPW;
    const int ncs = (int)(min<int64_t>((int64_t)(w0 + nw) * Sh::BPW, a.n_blocks) - cs0);
    const auto cr = rsrc(a.bcol + cs0, on ? (uint32_t)ncs * 4u : 0u);
#pragma unroll
    for (int k = 0; k < SM::NCR; ++k)
        in.colr[k] = __builtin_amdgcn_raw_buffer_load_b32(cr, (uint32_t)(lane * 4), 256 * k, kNT);
    const auto brr = rsrc(a.brow + d.i0, on ? (uint32_t)(nI + 1) * 4u : 0u);
    in.br[0] = __builtin_amdgcn_raw_buffer_load_b32(brr, (uint32_t)(lane * 4), 0, 0);
    in.br[1] = __builtin_amdgcn_raw_buffer_load_b32(brr, (uint32_t)(lane * 4), 256, 0);
    const auto mr = rsrc(a.mw + w0, on ? (uint32_t)nw * 8u : 0u);
    in.m = __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(mr, (uint32_t)(lane * 8), 0, kNT));
    const auto vr = rsrc(vals + abase, on ? (uint32_t)q_tail * 16u : 0u);
#pragma unroll
    for (int k = 0; k < KQ; ++k)
        chunk_to_lds(vr, s_vals + 64 * k * E, (uint32_t)(lane * 16), 1024 * k);
}

// The compute of a tile whose values are in s_vals (chunk order). prefetch()
// issues the next tile's loads (its values into s_vals once this tile's
// value reads are complete); it runs after this tile's gathers. The partials
// go to s_part.
template <class Sh, class T, int KQ, class F>
__device__ __forceinline__ void tile_run_lds(const SpmvArgs &a, const TileDesc &d, const TileNext<Sh, T, KQ> &in,
                                             __amdgpu_buffer_rsrc_t xr, int *s_brow, T *s_vals, double *s_part,
                                             const double *s_zero, F &&prefetch, YOut<T> *out) {
    using SM = WaveSmem<Sh, T, KQ>;
    constexpr int E = SM::E;
    const int lane = threadIdx.x & 63;
    const T *__restrict__ vals = static_cast<const T *>(a.vals);
    const int b0 = d.b0, b1 = d.b1, nv = d.nv;
    const int64_t abase = d.vbase & ~(int64_t)(E - 1);
    const int shift = (int)(d.vbase - abase);
    const int nq = (shift + nv + E - 1) / E;
    const int q_tail = (abase + (int64_t)nq * E > a.nnz) ? nq - 1 : nq;
    const int w0 = b0 / Sh::BPW;
    const int nw = (b1 > b0) ? ((b1 - 1) / Sh::BPW - w0 + 1) : 0;
    const int lo_slot = b0 - w0 * Sh::BPW;
    const uint64_t lo_mask = ~low_bits(lo_slot * Sh::RC);
    s_brow[lane] = in.br[0] - b0;
    s_brow[lane + 64] = in.br[1] - b0;
    // the array's last chunk may reach past nnz: its values are read one by
    // one (after the chunk loads have landed, which wrote zeros there)
    if (q_tail < nq && lane < E) {
        const int64_t g = abase + (int64_t)q_tail * E + lane;
        if (g < a.nnz) s_vals[q_tail * E + lane] = vals[g];
    }
    if (nw > 0) {
        constexpr int NWM = SM::NWMAX;
        constexpr int PPR = sizeof(T) == 8 ? 2 : 1;
        constexpr int W = Sh::C / PPR;
        const int slot = lane / Sh::RC;
        const int kcol = (lane % Sh::RC) % Sh::C;
        const char *__restrict__ bb = reinterpret_cast<const char *>(s_vals);
        const uint32_t zbyte = (uint32_t)(reinterpret_cast<const char *>(s_zero) - bb);
        int colj[NWM];
#pragma unroll
        for (int j = 0; j < NWM; ++j)
            colj[j] = __builtin_amdgcn_ds_bpermute(((j * Sh::BPW) % 64 + slot) * 4, in.colr[(j * Sh::BPW) / 64]);
        wave_sync();  // the tail values are in LDS
        // per word, in one pass: the x gather and the lane's value (the zero
        // slot where its bit is clear); words past the tile's last one are zero
        T xv[NWM], pv[NWM];
        uint32_t vbyte = (uint32_t)shift * (uint32_t)sizeof(T);
#pragma unroll
        for (int j = 0; j < NWM; ++j) {
            uint64_t m = readlane64(in.m, j);
            if (j == 0) m &= lo_mask;
            xv[j] = buf_load<T>(xr, pick(m, (uint32_t)(colj[j] + kcol) * (uint32_t)sizeof(T), 0xffffffffu));
            pv[j] = *reinterpret_cast<const T *>(bb + pick(m, lane_rank(m) * (uint32_t)sizeof(T) + vbyte, zbyte));
            vbyte += (uint32_t)__popcll(m) * (uint32_t)sizeof(T);
        }
        prefetch();
        double *__restrict__ mine = s_part + lane / W;
        const bool keeper = (lane % W) == 0;
#pragma unroll
        for (int j = 0; j < NWM; ++j) store_partial_at<Sh, T>(mine, keeper, j, pv[j] * xv[j]);
    } else {
        prefetch();
    }
    wave_sync();
    tile_sums<Sh, T, true>(a, d, lo_slot, w0, s_brow, s_part, out);
}

template <int R, int C, class T, int KQ>
__global__ __launch_bounds__(kThreads) void k_spmv_wave_pipe(SpmvArgs a) {
    using Sh = Shape<R, C>;
    using SM = WaveSmem<Sh, T, KQ>;
    __shared__ PipeSmem<Sh, T, KQ> sm[kWaves];
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int stride = (int)gridDim.x * kWaves;
    int t = (int)blockIdx.x * kWaves + wid;
    if (t >= a.n_tiles) return;
    const auto xr = rsrc(a.x, (uint32_t)(a.n_cols * (int64_t)sizeof(T)));
    PipeSmem<Sh, T, KQ> &S = sm[wid];
    if (lane_id() < 2) S.zero[lane_id()] = 0.0;
    TileDesc d = a.tiles[t];
    bool lng = d.b1 - d.b0 > SM::NB;
    TileNext<Sh, T, KQ> cur;
    tile_issue_lds<Sh, T, KQ>(a, d, cur, S.buf, !lng);
    int dn_raw = desc_lane(a, t + stride);   // all lanes 0 past the last tile
    // A tile's row results are stored after the next tile's loads have been
    // issued, so that the wait for those loads does not also wait for the
    // stores (memory operations are counted together, in issue order).
    const auto yr = rsrc(a.y, (uint32_t)a.n_rows * (uint32_t)sizeof(T));
    YOut<T> pend;
    pend.off[0] = pend.off[1] = 0xffffffffu;
    pend.val[0] = pend.val[1] = T(0);
    while (true) {
        wait_vm_all();  // this tile's streams and the next descriptor have landed
        const int tn = t + stride;
        const bool more = tn < a.n_tiles;
        const TileDesc dn = desc_from_lanes(dn_raw);
        const bool lngn = dn.b1 - dn.b0 > SM::NB;
        TileNext<Sh, T, KQ> nxt;
        int dnn_raw = 0;
        auto prefetch = [&]() {
            wait_lds_all();  // this tile's value reads are complete
            tile_issue_lds<Sh, T, KQ>(a, dn, nxt, S.buf, more && !lngn);
            dnn_raw = desc_lane(a, tn + stride);
            y_flush(yr, pend);  // the previous tile's rows
        };
        if (lng) {
            wave_long<Sh, T>(a, d.i0, d.b0, d.b1, d.vbase);
            prefetch();
            pend.off[0] = pend.off[1] = 0xffffffffu;
        } else {
            tile_run_lds<Sh, T, KQ>(a, d, cur, xr, S.brow, S.buf, S.part, S.zero, prefetch, &pend);
        }
        if (!more) {
            y_flush(yr, pend);
            break;
        }
        wave_sync();  // this tile's LDS reads are done before the next tile writes
        t = tn;
        d = dn;
        lng = lngn;
        cur = nxt;
        dn_raw = dnn_raw;
    }
}

// ---------------------------------------------------------------------------
// Mode 2, "test" tiles (Algorithm 2 of the paper, for the shapes whose block
// mask is one byte, beta(1,8) and beta(2,4)): a block holding a single value
// needs no expansion, its value goes straight to its row with one multiply,
// while the other blocks take the expanding path. On a wavefront:
//   S. lane = block (64 per round): the block's mask byte comes from its
//      word by a cross-lane move, a prefix count over the blocks gives each
//      block's first value; a single-value block's lane reads that value,
//      finds its column from the bit's position and gathers x; every other
//      block is appended to a compact list in LDS (mask, first value, slot,
//      column);
//   M. lane = mask bit of the compacted blocks (8 per 64-lane word, no lane
//      spent on single-value blocks): the value at the block's first value
//      plus the bit's rank, the x gather, and the lane sums per block row
//      into the (block, block row) partials;
//   then the row sums of the wavefront tiles. A tile holds up to NB2 blocks,
//   at most NM2 of them with several values, and at most the value buffer.
template <class Sh, class T, int KQ>
struct TestSmem {
    static constexpr int E = 16 / sizeof(T);
    static constexpr int NBUF = 64 * KQ * E;
    static constexpr int PPR = sizeof(T) == 8 ? 2 : 1;
    // the partial entries of every slot (up to 7 before the first block)
    // lie inside the value buffer, and 4 rounds of 64 lanes cover the slots
    static constexpr int NB2A = NBUF * (int)sizeof(T) / (Sh::R * PPR * 8) - 8;
    static constexpr int NB2 = NB2A < 248 ? NB2A : 248;
    static constexpr int NRS = (NB2 + 8 + 63) / 64;   // rounds of lane = block slot
    static constexpr int NM2 = 64;                    // blocks with several values per tile
    static constexpr int NWC = NM2 / 8;               // compacted mask words
    static_assert(Sh::R * Sh::C == 8, "test tiles are for the shapes with one-byte masks");
    T buf[NBUF];          // packed values, then the partials (double)
    int brow[128];
    double zero[2];
    uint32_t cpk[NM2];    // compacted blocks: mask | first value << 8 | slot << 20
    int32_t ccol[NM2];    // their columns
};

// One test tile on a wavefront (not a long one).
template <class Sh, class T, int KQ>
__device__ __forceinline__ void test_tile(const SpmvArgs &a, const TileDesc &d, TestSmem<Sh, T, KQ> &sm) {
    using SM = TestSmem<Sh, T, KQ>;
    constexpr int R = Sh::R, C = Sh::C;
    constexpr int E = SM::E;
    constexpr int PPR = SM::PPR;
    constexpr int W = C / PPR;            // lanes added into one partial
    const int lane = lane_id();
    const T *__restrict__ vals = static_cast<const T *>(a.vals);
    const int b0 = d.b0, b1 = d.b1, nv = d.nv, nI = d.i1 - d.i0;
    const int64_t abase = d.vbase & ~(int64_t)(E - 1);
    const int shift = (int)(d.vbase - abase);
    const int nq = (shift + nv + E - 1) / E;
    const int q_tail = (abase + (int64_t)nq * E > a.nnz) ? nq - 1 : nq;
    const int w0 = b0 / 8;
    const int lo_slot = b0 - w0 * 8;
    const int hi_slot = lo_slot + (b1 - b0);  // slots [lo_slot, hi_slot) are the tile's blocks
    const int nw = (b1 > b0) ? ((b1 - 1) / 8 - w0 + 1) : 0;
    // streams: block columns (slot lane + 64 k), interval pointers and mask
    // words (lane j: word j) into registers; the packed values into LDS
    const int cs0 = w0 * 8;
    const int ncs = (int)(min<int64_t>((int64_t)(w0 + nw) * 8, a.n_blocks) - cs0);
    const auto cr = rsrc(a.bcol + cs0, (uint32_t)(ncs > 0 ? ncs : 0) * 4u);
    int colr[SM::NRS];
#pragma unroll
    for (int k = 0; k < SM::NRS; ++k)
        colr[k] = __builtin_amdgcn_raw_buffer_load_b32(cr, (uint32_t)(lane * 4), 256 * k, kNT);
    const auto brr = rsrc(a.brow + d.i0, (uint32_t)(nI + 1) * 4u);
    const int br0 = __builtin_amdgcn_raw_buffer_load_b32(brr, (uint32_t)(lane * 4), 0, 0);
    const int br1 = __builtin_amdgcn_raw_buffer_load_b32(brr, (uint32_t)(lane * 4), 256, 0);
    const auto mr = rsrc(a.mw + w0, (uint32_t)nw * 8u);
    const uint64_t mword =
        __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(mr, (uint32_t)(lane * 8), 0, kNT));
    values_to_lds<T, KQ>(rsrc(vals + abase, (uint32_t)q_tail * 16u), sm.buf);
    sm.brow[lane] = br0 - b0;
    sm.brow[lane + 64] = br1 - b0;
    if (lane < 2) sm.zero[lane] = 0.0;
    wait_vm_all();
    if (q_tail < nq && lane < E) {
        const int64_t gi = abase + (int64_t)q_tail * E + lane;
        if (gi < a.nnz) sm.buf[q_tail * E + lane] = vals[gi];
    }
    wave_sync();
    const auto xr = rsrc(a.x, (uint32_t)(a.n_cols * (int64_t)sizeof(T)));
    const char *__restrict__ bb = reinterpret_cast<const char *>(sm.buf);
    const uint32_t zbyte = (uint32_t)(reinterpret_cast<const char *>(sm.zero) - bb);
    const uint32_t lo32 = (uint32_t)mword, hi32 = (uint32_t)(mword >> 32);

    // S. lane = block slot
    T xs[SM::NRS], vs[SM::NRS];
    int srho[SM::NRS];
    uint64_t single_m[SM::NRS];
    int vcarry = 0, mcarry = 0;
#pragma unroll
    for (int k = 0; k < SM::NRS; ++k) {
        const int sl = lane + 64 * k;
        // the word of slot sl is held by lane sl / 8 (lanes 8 k .. 8 k + 7)
        const int src = (lane / 8 + 8 * k) * 4;
        const uint32_t wlo = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)lo32);
        const uint32_t whi = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)hi32);
        const int sh = (sl % 8) * 8;
        uint32_t mk = (sh < 32 ? (wlo >> sh) : (whi >> (sh - 32))) & 0xffu;
        mk = (sl >= lo_slot && sl < hi_slot) ? mk : 0u;
        const int pc = __popc(mk);
        const int incl = wave_scan_dpp(pc);
        const int voff = vcarry + incl - pc;           // the block's first value in the tile
        vcarry += __builtin_amdgcn_readlane(incl, 63);
        const int tb = __builtin_ctz(mk | 0x100u);     // position of a single block's bit
        srho[k] = tb / C;
        const uint64_t sb = ballot64(pc == 1);
        single_m[k] = sb;
        xs[k] = buf_load<T>(xr, pick(sb, (uint32_t)(colr[k] + tb % C) * (uint32_t)sizeof(T), 0xffffffffu));
        vs[k] = *reinterpret_cast<const T *>(bb + pick(sb, (uint32_t)(shift + voff) * (uint32_t)sizeof(T), zbyte));
        const uint64_t mb = ballot64(pc >= 2);
        const int mr_ = mcarry + (int)lane_rank(mb);
        if (pc >= 2) {
            sm.cpk[mr_] = mk | ((uint32_t)voff << 8) | ((uint32_t)sl << 20);
            sm.ccol[mr_] = colr[k];
        }
        mcarry += __popcll(mb);
    }
    wave_sync();  // the compact list is written

    // M. lane = mask bit of the compacted blocks
    const int bit = lane % 8;
    const int kc = bit % C;
    const uint32_t below = (1u << bit) - 1u;
    T xm[SM::NWC], vm[SM::NWC];
#pragma unroll
    for (int w = 0; w < SM::NWC; ++w) {
        const int cb = 8 * w + lane / 8;
        const bool in = cb < mcarry;
        const uint32_t pk = in ? sm.cpk[cb] : 0u;
        const int cc = in ? sm.ccol[cb] : 0;
        const uint64_t sb = ballot64((pk >> bit) & 1u);
        const uint32_t vpos = (uint32_t)shift + ((pk >> 8) & 0xfffu) + (uint32_t)__popc(pk & 0xffu & below);
        xm[w] = buf_load<T>(xr, pick(sb, (uint32_t)(cc + kc) * (uint32_t)sizeof(T), 0xffffffffu));
        vm[w] = *reinterpret_cast<const T *>(bb + pick(sb, vpos * (uint32_t)sizeof(T), zbyte));
    }
    wave_sync();  // every value is read before the partials overwrite them

    double *__restrict__ part = reinterpret_cast<double *>(sm.buf);
    // single-value blocks: the product in its row's first entry, zeros in
    // the block's other entries
#pragma unroll
    for (int k = 0; k < SM::NRS; ++k) {
        if ((single_m[k] >> lane) & 1ull) {
            const int sl = lane + 64 * k;
            const double pr = (double)(vs[k] * xs[k]);
#pragma unroll
            for (int e = 0; e < R * PPR; ++e) part[sl * R * PPR + e] = e == srho[k] * PPR ? pr : 0.0;
        }
    }
    // compacted blocks: lane sums over each block row's W lanes
    const bool keeper = (lane % W) == 0;
    const int rho = bit / C, h = kc / W;
#pragma unroll
    for (int w = 0; w < SM::NWC; ++w) {
        T p = vm[w] * xm[w];
        if constexpr (sizeof(T) == 8) {
            p += dpp_f64<0xb1>(p);                          // quad_perm [1,0,3,2]
            if constexpr (W == 4) p += dpp_f64<0x4e>(p);    // quad_perm [2,3,0,1]
        } else {
            p = row_group_sum<C>(p);
        }
        const int cb = 8 * w + lane / 8;
        if (keeper && cb < mcarry) {
            const int sl = (int)(sm.cpk[cb] >> 20);
            part[(sl * R + rho) * PPR + h] = (double)p;
        }
    }
    wave_sync();
    tile_sums<Sh, T>(a, d, lo_slot, w0, sm.brow, part);
}

template <int R, int C, class T, int KQ>
__global__ __launch_bounds__(kThreads) void k_spmv_test(SpmvArgs a) {
    using Sh = Shape<R, C>;
    __shared__ TestSmem<Sh, T, KQ> smem[kWaves];
    int g = blockIdx.x;
    if (a.xcd_remap) g = (int)(blockIdx.x & 7u) * a.tiles_per_xcd + (int)(blockIdx.x >> 3);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = g * kWaves + wid;
    if (t >= a.n_tiles) return;
    const TileDesc d = a.tiles[t];
    if (d.reserved & 1) {                 // one interval beyond a test tile's limits
        wave_long<Sh, T>(a, d.i0, d.b0, d.b1, d.vbase);
        return;
    }
    test_tile<Sh, T, KQ>(a, d, smem[wid]);
}

template <int R, int C, class T>
spc_status launch_test(int kq, int cu_groups, dim3 grid, const SpmvArgs &a, hipStream_t stream) {
    const dim3 blk(kThreads);
    switch (kq) {
    case 2: return launch_capped(k_spmv_test<R, C, T, 2>, cu_groups, grid, blk, stream, a);
    case 6: return launch_capped(k_spmv_test<R, C, T, 6>, cu_groups, grid, blk, stream, a);
    case 8: return launch_capped(k_spmv_test<R, C, T, 8>, cu_groups, grid, blk, stream, a);
    default: return launch_capped(k_spmv_test<R, C, T, 4>, cu_groups, grid, blk, stream, a);
    }
}

// Test tiles exist for the two shapes with one-byte masks only.
spc_status launch_test_shape(int shape, int dtype, int kq, int cu_groups, dim3 grid, const SpmvArgs &a,
                             hipStream_t stream) {
    if (shape == 0)
        return dtype == SPC_F64 ? launch_test<1, 8, double>(kq, cu_groups, grid, a, stream)
                                : launch_test<1, 8, float>(kq, cu_groups, grid, a, stream);
    if (shape == 1)
        return dtype == SPC_F64 ? launch_test<2, 4, double>(kq, cu_groups, grid, a, stream)
                                : launch_test<2, 4, float>(kq, cu_groups, grid, a, stream);
    set_error("test tiles are for beta(1,8) and beta(2,4)");
    return SPC_ERR_UNSUPPORTED_SHAPE;
}

// Batched test tiles: TileDesc::reserved holds (matrix index << 1) | long
// flag. A wavefront loops over the tiles t, t + S, ... (S = 4 x grid), so a
// grid smaller than the list is persistent.
template <int R, int C, class T, int KQ>
__global__ __launch_bounds__(kThreads) void k_spmv_batched_test(const BatchMat *__restrict__ mats,
                                                                const TileDesc *__restrict__ tiles, int64_t n_tiles,
                                                                int accumulate) {
    using Sh = Shape<R, C>;
    __shared__ TestSmem<Sh, T, KQ> smem[kWaves];
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t step = (int64_t)gridDim.x * kWaves;
    for (int64_t t = (int64_t)blockIdx.x * kWaves + wid; t < n_tiles; t += step) {
        const TileDesc d = tiles[t];
        const SpmvArgs a = batch_args(mats[d.reserved >> 1], tiles, accumulate);
        wave_sync();  // the previous tile's LDS reads are done before this tile writes
        if (d.reserved & 1) wave_long<Sh, T>(a, d.i0, d.b0, d.b1, d.vbase);
        else test_tile<Sh, T, KQ>(a, d, smem[wid]);
    }
}

template <int R, int C, class T>
void launch_batched_test(int kq, unsigned grid, const BatchMat *d_mats, const TileDesc *d_tiles, int64_t n_tiles,
                         int accumulate, hipStream_t stream) {
    switch (kq) {
    case 2:
        hipLaunchKernelGGL((k_spmv_batched_test<R, C, T, 2>), dim3(grid), dim3(kThreads), 0, stream, d_mats, d_tiles,
                           n_tiles, accumulate);
        break;
    case 6:
        hipLaunchKernelGGL((k_spmv_batched_test<R, C, T, 6>), dim3(grid), dim3(kThreads), 0, stream, d_mats, d_tiles,
                           n_tiles, accumulate);
        break;
    case 8:
        hipLaunchKernelGGL((k_spmv_batched_test<R, C, T, 8>), dim3(grid), dim3(kThreads), 0, stream, d_mats, d_tiles,
                           n_tiles, accumulate);
        break;
    default:
        hipLaunchKernelGGL((k_spmv_batched_test<R, C, T, 4>), dim3(grid), dim3(kThreads), 0, stream, d_mats, d_tiles,
                           n_tiles, accumulate);
        break;
    }
}

// Batched block-row-lane (mode 3) and value-lane (mode 4) tiles:
// TileDesc::reserved holds the matrix index; an interval beyond a tile's
// values or blocks takes the long path, as in the single-matrix kernels. A
// wavefront loops over the tiles t, t + S, ... (S = 4 x grid).
template <int R, int C, class T, int KQ>
__global__ __launch_bounds__(kThreads) void k_spmv_batched_brow(const BatchMat *__restrict__ mats,
                                                                const TileDesc *__restrict__ tiles, int64_t n_tiles,
                                                                int accumulate) {
    using Sh = Shape<R, C>;
    using SM = BrowSmem<Sh, T, KQ>;
    __shared__ SM smem[kWaves];
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t step = (int64_t)gridDim.x * kWaves;
    for (int64_t t = (int64_t)blockIdx.x * kWaves + wid; t < n_tiles; t += step) {
        const TileDesc d = tiles[t];
        const SpmvArgs a = batch_args(mats[d.reserved], tiles, accumulate);
        wave_sync();  // the previous tile's LDS reads are done before this tile writes
        if (d.b1 - d.b0 > SM::NBX || d.nv > SM::VCAP) {
            wave_long<Sh, T>(a, d.i0, d.b0, d.b1, d.vbase);
        } else {
            const auto xr = rsrc(a.x, (uint32_t)(a.n_cols * (int64_t)sizeof(T)));
            brow_tile<Sh, T, KQ>(a, d, xr, smem[wid]);
        }
    }
}

template <class T, int KQ>
__global__ __launch_bounds__(kThreads) void k_spmv_batched_vlane(const BatchMat *__restrict__ mats,
                                                                 const TileDesc *__restrict__ tiles, int64_t n_tiles,
                                                                 int accumulate) {
    using Sh = Shape<1, 8>;
    using SM = VlaneSmem<Sh, T, KQ>;
    __shared__ SM smem[kWaves];
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t step = (int64_t)gridDim.x * kWaves;
    for (int64_t t = (int64_t)blockIdx.x * kWaves + wid; t < n_tiles; t += step) {
        const TileDesc d = tiles[t];
        const SpmvArgs a = batch_args(mats[d.reserved], tiles, accumulate);
        wave_sync();
        if (d.b1 - d.b0 > SM::NBX || d.nv > SM::VCAP) {
            wave_long<Sh, T>(a, d.i0, d.b0, d.b1, d.vbase);
        } else {
            const auto xr = rsrc(a.x, (uint32_t)(a.n_cols * (int64_t)sizeof(T)));
            vlane_tile<Sh, T, KQ>(a, d, xr, smem[wid]);
        }
    }
}

template <int R, int C, class T>
void launch_batched_brow(int kq, unsigned grid, const BatchMat *d_mats, const TileDesc *d_tiles, int64_t n_tiles,
                         int accumulate, hipStream_t stream) {
    const dim3 g(grid), b(kThreads);
    switch (kq) {
    case 2: hipLaunchKernelGGL((k_spmv_batched_brow<R, C, T, 2>), g, b, 0, stream, d_mats, d_tiles, n_tiles, accumulate); break;
    case 6: hipLaunchKernelGGL((k_spmv_batched_brow<R, C, T, 6>), g, b, 0, stream, d_mats, d_tiles, n_tiles, accumulate); break;
    case 8: hipLaunchKernelGGL((k_spmv_batched_brow<R, C, T, 8>), g, b, 0, stream, d_mats, d_tiles, n_tiles, accumulate); break;
    default: hipLaunchKernelGGL((k_spmv_batched_brow<R, C, T, 4>), g, b, 0, stream, d_mats, d_tiles, n_tiles, accumulate); break;
    }
}

template <class T>
void launch_batched_vlane(int kq, unsigned grid, const BatchMat *d_mats, const TileDesc *d_tiles, int64_t n_tiles,
                          int accumulate, hipStream_t stream) {
    const dim3 g(grid), b(kThreads);
    switch (kq) {
    case 2: hipLaunchKernelGGL((k_spmv_batched_vlane<T, 2>), g, b, 0, stream, d_mats, d_tiles, n_tiles, accumulate); break;
    case 6: hipLaunchKernelGGL((k_spmv_batched_vlane<T, 6>), g, b, 0, stream, d_mats, d_tiles, n_tiles, accumulate); break;
    case 8: hipLaunchKernelGGL((k_spmv_batched_vlane<T, 8>), g, b, 0, stream, d_mats, d_tiles, n_tiles, accumulate); break;
    default: hipLaunchKernelGGL((k_spmv_batched_vlane<T, 4>), g, b, 0, stream, d_mats, d_tiles, n_tiles, accumulate); break;
    }
}

template <int R, int C, class T>
spc_status launch_wg(int tb, dim3 grid, const SpmvArgs &a, hipStream_t stream) {
    switch (tb) {
    case 1024: hipLaunchKernelGGL((k_spmv_wg<R, C, T, 1024>), grid, dim3(kThreads), 0, stream, a); break;
    case 2048: hipLaunchKernelGGL((k_spmv_wg<R, C, T, 2048>), grid, dim3(kThreads), 0, stream, a); break;
    case 3072: hipLaunchKernelGGL((k_spmv_wg<R, C, T, 3072>), grid, dim3(kThreads), 0, stream, a); break;
    default: hipLaunchKernelGGL((k_spmv_wg<R, C, T, 4032>), grid, dim3(kThreads), 0, stream, a); break;
    }
    SPC_HIP(hipGetLastError());
    return SPC_OK;
}

template <int R, int C, class T>
spc_status launch_wave_pipe(int kq, dim3 grid, const SpmvArgs &a, hipStream_t stream) {
    switch (kq) {
    case 2: hipLaunchKernelGGL((k_spmv_wave_pipe<R, C, T, 2>), grid, dim3(kThreads), 0, stream, a); break;
    case 6: hipLaunchKernelGGL((k_spmv_wave_pipe<R, C, T, 6>), grid, dim3(kThreads), 0, stream, a); break;
    case 8: hipLaunchKernelGGL((k_spmv_wave_pipe<R, C, T, 8>), grid, dim3(kThreads), 0, stream, a); break;
    default: hipLaunchKernelGGL((k_spmv_wave_pipe<R, C, T, 4>), grid, dim3(kThreads), 0, stream, a); break;
    }
    SPC_HIP(hipGetLastError());
    return SPC_OK;
}

// Workgroups of the pipelined kernel that are resident at once on the device.
template <int R, int C, class T>
spc_status resident_groups(int kq, int *out) {
    const void *f = kq == 2   ? reinterpret_cast<const void *>(k_spmv_wave_pipe<R, C, T, 2>)
                    : kq == 6 ? reinterpret_cast<const void *>(k_spmv_wave_pipe<R, C, T, 6>)
                    : kq == 8 ? reinterpret_cast<const void *>(k_spmv_wave_pipe<R, C, T, 8>)
                              : reinterpret_cast<const void *>(k_spmv_wave_pipe<R, C, T, 4>);
    int per_cu = 0, dev = 0, cus = 0;
    SPC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kThreads, 0));
    SPC_HIP(hipGetDevice(&dev));
    SPC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    *out = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
    return SPC_OK;
}

template <int R, int C, class T>
spc_status launch_wave2(int kq, int cu_groups, dim3 grid, const SpmvArgs &a, hipStream_t stream) {
    const dim3 blk(kThreads);
    switch (kq) {
    case 2: return launch_capped(k_spmv_wave2<R, C, T, 2>, cu_groups, grid, blk, stream, a);
    case 6: return launch_capped(k_spmv_wave2<R, C, T, 6>, cu_groups, grid, blk, stream, a);
    case 8: return launch_capped(k_spmv_wave2<R, C, T, 8>, cu_groups, grid, blk, stream, a);
    default: return launch_capped(k_spmv_wave2<R, C, T, 4>, cu_groups, grid, blk, stream, a);
    }
}

template <int R, int C, class T>
spc_status launch_wave(int kq, int cu_groups, dim3 grid, const SpmvArgs &a, hipStream_t stream) {
    const dim3 blk(kThreads);
    switch (kq) {
    case 2: return launch_capped(k_spmv_wave<R, C, T, 2>, cu_groups, grid, blk, stream, a);
    case 6: return launch_capped(k_spmv_wave<R, C, T, 6>, cu_groups, grid, blk, stream, a);
    case 8: return launch_capped(k_spmv_wave<R, C, T, 8>, cu_groups, grid, blk, stream, a);
    default: return launch_capped(k_spmv_wave<R, C, T, 4>, cu_groups, grid, blk, stream, a);
    }
}

template <int R, int C, class T>
spc_status launch_brow(int kq, int cu_groups, dim3 grid, const SpmvArgs &a, hipStream_t stream) {
    const dim3 blk(kThreads);
    switch (kq) {
    case 2: return launch_capped(k_spmv_brow<R, C, T, 2>, cu_groups, grid, blk, stream, a);
    case 6: return launch_capped(k_spmv_brow<R, C, T, 6>, cu_groups, grid, blk, stream, a);
    case 8: return launch_capped(k_spmv_brow<R, C, T, 8>, cu_groups, grid, blk, stream, a);
    default: return launch_capped(k_spmv_brow<R, C, T, 4>, cu_groups, grid, blk, stream, a);
    }
}

template <class T>
spc_status launch_vlane(int kq, int cu_groups, dim3 grid, const SpmvArgs &a, hipStream_t stream) {
    const dim3 blk(kThreads);
    switch (kq) {
    case 2: return launch_capped(k_spmv_vlane<T, 2>, cu_groups, grid, blk, stream, a);
    case 6: return launch_capped(k_spmv_vlane<T, 6>, cu_groups, grid, blk, stream, a);
    case 8: return launch_capped(k_spmv_vlane<T, 8>, cu_groups, grid, blk, stream, a);
    default: return launch_capped(k_spmv_vlane<T, 4>, cu_groups, grid, blk, stream, a);
    }
}

}  // namespace

spc_status batched_launch(int dtype, int kq, const BatchMat *d_mats, const TileDesc *d_tiles, int64_t n_tiles,
                          int accumulate, int grid_blocks, int single_shape, hipStream_t stream) {
    if (n_tiles == 0) return SPC_OK;
    const int64_t groups = div_up(n_tiles, kWaves);
    const unsigned grid = (unsigned)(grid_blocks > 0 && grid_blocks < groups ? grid_blocks : groups);
    return with_dtype(dtype, [&](auto tv) -> spc_status {
        using T = decltype(tv);
        if (single_shape >= 0) {
            const bool persist = grid < groups;
            switch (single_shape) {
            case 0: launch_batched_fixed<0, T>(kq, grid, persist, d_mats, d_tiles, n_tiles, accumulate, stream); break;
            case 1: launch_batched_fixed<1, T>(kq, grid, persist, d_mats, d_tiles, n_tiles, accumulate, stream); break;
            case 2: launch_batched_fixed<2, T>(kq, grid, persist, d_mats, d_tiles, n_tiles, accumulate, stream); break;
            case 3: launch_batched_fixed<3, T>(kq, grid, persist, d_mats, d_tiles, n_tiles, accumulate, stream); break;
            case 4: launch_batched_fixed<4, T>(kq, grid, persist, d_mats, d_tiles, n_tiles, accumulate, stream); break;
            default: launch_batched_fixed<5, T>(kq, grid, persist, d_mats, d_tiles, n_tiles, accumulate, stream);
                break;
            }
            SPC_HIP(hipGetLastError());
            return SPC_OK;
        }
        const bool persist = grid < groups;
        auto go = [&](auto kq_c) {
            constexpr int KQ = decltype(kq_c)::value;
            if (persist)
                hipLaunchKernelGGL((k_spmv_batched<T, KQ, true>), dim3(grid), dim3(kThreads), 0, stream, d_mats,
                                   d_tiles, n_tiles, accumulate);
            else
                hipLaunchKernelGGL((k_spmv_batched<T, KQ, false>), dim3(grid), dim3(kThreads), 0, stream, d_mats,
                                   d_tiles, n_tiles, accumulate);
        };
        switch (kq) {
        case 2: go(std::integral_constant<int, 2>{}); break;
        case 6: go(std::integral_constant<int, 6>{}); break;
        case 8: go(std::integral_constant<int, 8>{}); break;
        default: go(std::integral_constant<int, 4>{}); break;
        }
        SPC_HIP(hipGetLastError());
        return SPC_OK;
    });
}

spc_status batched_launch_test(int dtype, int shape, int kq, const BatchMat *d_mats, const TileDesc *d_tiles,
                               int64_t n_tiles, int accumulate, int grid_blocks, hipStream_t stream) {
    SPC_REQUIRE(shape == 0 || shape == 1, SPC_ERR_UNSUPPORTED_SHAPE, "test tiles are for beta(1,8) and beta(2,4)");
    if (n_tiles == 0) return SPC_OK;
    const int64_t groups = div_up(n_tiles, kWaves);
    const unsigned grid = (unsigned)(grid_blocks > 0 && grid_blocks < groups ? grid_blocks : groups);
    return with_dtype(dtype, [&](auto tv) -> spc_status {
        using T = decltype(tv);
        if (shape == 0) launch_batched_test<1, 8, T>(kq, grid, d_mats, d_tiles, n_tiles, accumulate, stream);
        else launch_batched_test<2, 4, T>(kq, grid, d_mats, d_tiles, n_tiles, accumulate, stream);
        SPC_HIP(hipGetLastError());
        return SPC_OK;
    });
}

spc_status batched_launch_lanes(int dtype, int mode, int shape, int kq, const BatchMat *d_mats,
                                const TileDesc *d_tiles, int64_t n_tiles, int accumulate, int grid_blocks,
                                hipStream_t stream) {
    SPC_REQUIRE(mode == 3 || (mode == 4 && shape == 0), SPC_ERR_UNSUPPORTED_SHAPE,
                "batched lanes: mode 3, or mode 4 for beta(1,8)");
    if (n_tiles == 0) return SPC_OK;
    const int64_t groups = div_up(n_tiles, kWaves);
    const unsigned grid = (unsigned)(grid_blocks > 0 && grid_blocks < groups ? grid_blocks : groups);
    return with_dtype(dtype, [&](auto tv) -> spc_status {
        using T = decltype(tv);
        if (mode == 4) {
            launch_batched_vlane<T>(kq, grid, d_mats, d_tiles, n_tiles, accumulate, stream);
        } else {
            with_shape(shape, [&](auto sh) {
                using Sh = decltype(sh);
                launch_batched_brow<Sh::R, Sh::C, T>(kq, grid, d_mats, d_tiles, n_tiles, accumulate, stream);
                return 0;
            });
        }
        SPC_HIP(hipGetLastError());
        return SPC_OK;
    });
}

spc_status spmv_resident_groups(int shape, int dtype, int kq, int *out) {
    return with_shape(shape, [&](auto sh) {
        using Sh = decltype(sh);
        return with_dtype(dtype, [&](auto tv) {
            using T = decltype(tv);
            return resident_groups<Sh::R, Sh::C, T>(kq, out);
        });
    });
}

// Mode 0 loads a tile's interval pointers two per lane (up to 128, the end pointer
// included) and takes up to 128 (interval, block row) pairs, two per lane.
int spmv_max_intervals_per_tile(int r, int mode) { return mode == 0 ? (r == 1 ? 127 : 128 / r) : kThreads / r; }

// Blocks a test tile (mode 2) may hold, of which at most 64 with several
// values; 0 for shapes without test tiles.
int test_tile_blocks(int shape, int dtype, int kq) {
    auto nb = [&](auto sh, auto tv) -> int {
        using Sh = decltype(sh);
        using T = decltype(tv);
        switch (kq) {
        case 2: return TestSmem<Sh, T, 2>::NB2;
        case 6: return TestSmem<Sh, T, 6>::NB2;
        case 8: return TestSmem<Sh, T, 8>::NB2;
        default: return TestSmem<Sh, T, 4>::NB2;
        }
    };
    if (shape == 0) return dtype == SPC_F64 ? nb(Shape<1, 8>{}, double{}) : nb(Shape<1, 8>{}, float{});
    if (shape == 1) return dtype == SPC_F64 ? nb(Shape<2, 4>{}, double{}) : nb(Shape<2, 4>{}, float{});
    return 0;
}

// Tile capacity in mask bits for a mode and a chunk count (mode 0) or the
// workgroup tile size (mode 1).
// Blocks a block-row-lane tile (mode 3) may hold.
int brow_tile_blocks(int shape, int dtype, int kq) {
    return with_shape(shape, [&](auto sh) {
        using Sh = decltype(sh);
        auto nb = [&](auto tv) -> int {
            using T = decltype(tv);
            switch (kq) {
            case 2: return BrowSmem<Sh, T, 2>::NBX;
            case 6: return BrowSmem<Sh, T, 6>::NBX;
            case 8: return BrowSmem<Sh, T, 8>::NBX;
            default: return BrowSmem<Sh, T, 4>::NBX;
            }
        };
        return dtype == SPC_F64 ? nb(0.0) : nb(0.f);
    });
}

int wave_tile_bits(int dtype, int kq) {
    const int E = dtype == SPC_F64 ? 2 : 4;
    return (64 * kq - 1) * E;
}

spc_status spmv_launch(const spc_beta_view *A, const spc_plan *P, const void *x, void *y, int accumulate,
                       hipStream_t stream) {
    SpmvArgs a;
    a.brow = A->block_rowptr;
    a.bcol = A->block_colidx;
    a.mw = static_cast<const uint64_t *>(A->block_masks);
    a.vals = A->values;
    a.x = x;
    a.y = y;
    a.tiles = P->d_tiles;
    a.n_rows = A->n_rows;
    a.nnz = A->nnz;
    a.n_blocks = A->n_blocks;
    a.n_cols = A->n_cols;
    a.n_tiles = (int32_t)P->n_tiles;
    a.accumulate = accumulate;
    a.xcd_remap = P->xcd_remap;
    // Wavefront tiles read values with 16-byte loads and address x with 32-bit
    // byte offsets, so they need a 16-byte aligned values array and x under
    // 4 GiB; otherwise the same tiles run as workgroup tiles (any workgroup
    // tile size at least as large as the plan's tiles works).
    const bool aligned = (reinterpret_cast<uintptr_t>(A->values) & 15u) == 0;
    const size_t es = A->dtype == SPC_F64 ? 8 : 4;
    const bool x32 = (uint64_t)A->n_cols * es < 0xf0000000ull;    // x addressed with 32-bit offsets
    const bool wave = P->mode != 1 && aligned && x32;
    const int wg_bits = P->mode == 1                   ? P->tile_bits
                        : (P->mode == 3 || P->mode == 4) ? 4032
                                                         : (P->tile_bits <= 1024 ? 1024 : 2048);
    const bool pair = wave && P->mode == 0 && P->wave_tiles == 2 && !P->pipeline;
    const int64_t groups = wave ? div_up(pair ? div_up(P->n_tiles, 2) : P->n_tiles, kWaves) : P->n_tiles;
    a.tiles_per_xcd = (int32_t)div_up(groups, 8);
    dim3 grid(P->xcd_remap ? (unsigned)(8 * a.tiles_per_xcd) : (unsigned)groups);
    // the pipelined kernel reads descriptors with 32-bit byte offsets
    // and addresses y with 32-bit byte offsets
    const bool pipe = wave && P->pipeline && P->resident > 0 && P->n_tiles < ((int64_t)1 << 27) &&
                      (uint64_t)A->n_rows * es < 0xf0000000ull;
    if (pipe) grid = dim3((unsigned)(groups < P->resident ? groups : (int64_t)P->resident));
    if (wave && P->mode == 2) return launch_test_shape(P->shape, A->dtype, P->kq, P->cu_groups, grid, a, stream);
    if (wave && P->mode == 4)
        return A->dtype == SPC_F64 ? launch_vlane<double>(P->kq, P->cu_groups, grid, a, stream)
                                   : launch_vlane<float>(P->kq, P->cu_groups, grid, a, stream);
    return with_shape(P->shape, [&](auto sh) {
        using Sh = decltype(sh);
        return with_dtype(A->dtype, [&](auto tv) {
            using T = decltype(tv);
            if (!wave) return launch_wg<Sh::R, Sh::C, T>(wg_bits, grid, a, stream);
            if (P->mode == 3) return launch_brow<Sh::R, Sh::C, T>(P->kq, P->cu_groups, grid, a, stream);
            if (pipe) return launch_wave_pipe<Sh::R, Sh::C, T>(P->kq, grid, a, stream);
            if (pair) return launch_wave2<Sh::R, Sh::C, T>(P->kq, P->cu_groups, grid, a, stream);
            return launch_wave<Sh::R, Sh::C, T>(P->kq, P->cu_groups, grid, a, stream);
        });
    });
}

}  // namespace spc
