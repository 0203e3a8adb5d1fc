// Y = A X for k right-hand sides over beta(r,c) (X, Y row-major, the k
// values of one row contiguous), on the wavefront tiles of a mode-0 plan.
//
// The matrix is streamed once for all k columns: a tile's values, columns,
// masks and interval pointers are read as in the single-vector kernel, and
// each lane keeps the value of its mask bit for every word of the tile. The
// k columns are then taken one after the other, each like one single-vector
// product over the tile (all x gathers of the tile in flight together, each
// block row's products added across lanes into one partial, two for FP64, in
// LDS, L lanes per row). Row sums are formed in double precision and written once
// per row and column.
//
// An interval with more blocks than a tile holds is run by one wavefront
// with lane = mask bit throughout, each lane keeping k running sums.
//
// Row path (wide right-hand sides, k x sizeof(T) >= 64 bytes per row): the
// tile's values and columns are first sorted by row in LDS (a prefix of
// each block row's value counts over the tile's blocks gives every value
// its place), then Q lanes take one row, lane g gathering the 16-byte
// column group g of each X row the row touches and keeping the group's
// sums; the Q lanes of a row store the whole Y row with one instruction.
// Every X row is fetched in full by one instruction and every Y row is
// written once.
#include "common.hpp"
#include "wave_common.hpp"

namespace spc {
namespace {

using namespace dev;

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kMaxK = 16;

struct SpmmArgs {
    const int32_t *brow;
    const int32_t *bcol;
    const uint64_t *mw;
    const void *vals;
    const void *X;
    void *Y;
    const TileDesc *tiles;
    int64_t n_rows, n_cols, nnz, n_blocks;
    int64_t ldx, ldy;
    int32_t k;
    int32_t wide;        // columns taken G = 16 / sizeof(T) at a time (see spmm_tile)
    int32_t n_tiles;
    int32_t accumulate;
    int32_t xcd_remap;
    int32_t tiles_per_xcd;
    int32_t lgq;         // row path: log2 of the lanes per row
};

template <class Sh, class T, int KQ>
struct SpmmSmem {
    static constexpr int E = 16 / sizeof(T);
    static constexpr int WB = (64 * KQ - 1) * E;
    static constexpr int NB = WB / Sh::RC;
    static constexpr int NWMAX = NB / Sh::BPW + 2;
    static constexpr int NCR = (NWMAX * Sh::BPW + 63) / 64;
    static constexpr int NBUF = 64 * KQ * E;
    // (block, block row) partials of the tile's words, G = E columns each
    static constexpr int PPR = sizeof(T) == 8 ? 2 : 1;   // partials per (block, block row)
    static constexpr int NPART = NWMAX * (64 / Sh::C) * PPR * E;
    static constexpr int NALL = NPART > NBUF ? NPART : NBUF;
    int brow[128];             // tile-relative interval pointers (up to 127 intervals)
    T buf[NALL];               // packed values, then the partials of a column group
};

// One tile, all k columns. The tile's streams are read once; every lane
// keeps the values of its mask bits and their X row offsets in registers;
// then for each column q the x gathers of all words are issued together,
// the products go to LDS in packed order and L lanes per (interval, block
// row) add them, as in the single-vector kernel.
template <class Sh, class T, int KQ>
__device__ void spmm_tile(const SpmmArgs &a, const TileDesc &d, __amdgpu_buffer_rsrc_t xr,
                          SpmmSmem<Sh, T, KQ> &sm) {
    using SM = SpmmSmem<Sh, T, KQ>;
    constexpr int E = SM::E;
    constexpr int NWM = SM::NWMAX;
    static_assert(NWM <= 64, "the masks array is padded for 64 words read past its end");
    using V4 = __attribute__((ext_vector_type(4))) unsigned int;
    const int lane = threadIdx.x & 63;
    const T *__restrict__ vals = static_cast<const T *>(a.vals);
    const int b0 = d.b0, b1 = d.b1, nv = d.nv, nI = d.i1 - d.i0;
    const int64_t abase = d.vbase & ~(int64_t)(E - 1);
    const int shift = (int)(d.vbase - abase);
    const int nq = (shift + nv + E - 1) / E;
    const int q_tail = (abase + (int64_t)nq * E > a.nnz) ? nq - 1 : nq;
    const int w0 = b0 / Sh::BPW;
    const int nw = (b1 > b0) ? ((b1 - 1) / Sh::BPW - w0 + 1) : 0;
    const int lo_slot = b0 - w0 * Sh::BPW;
    const uint64_t lo_mask = ~low_bits(lo_slot * Sh::RC);
    const int cs0 = w0 * Sh::BPW;
    const int ncs = (int)(min<int64_t>((int64_t)(w0 + nw) * Sh::BPW, a.n_blocks) - cs0);

    // 1. streams (buffer loads, unguarded), metadata into LDS
    const auto cr = rsrc(a.bcol + cs0, (uint32_t)ncs * 4u);
    int colr[SM::NCR];
#pragma unroll
    for (int k = 0; k < SM::NCR; ++k)
        colr[k] = __builtin_amdgcn_raw_buffer_load_b32(cr, (uint32_t)(lane * 4), 256 * k, kNT);
    const auto brr = rsrc(a.brow + d.i0, (uint32_t)(nI + 1) * 4u);
    const int br0 = __builtin_amdgcn_raw_buffer_load_b32(brr, (uint32_t)(lane * 4), 0, 0);
    const int br1 = __builtin_amdgcn_raw_buffer_load_b32(brr, (uint32_t)(lane * 4), 256, 0);
    const auto vr = rsrc(vals + abase, (uint32_t)q_tail * 16u);
    V4 ch[KQ];
#pragma unroll
    for (int k = 0; k < KQ; ++k)
        ch[k] = __builtin_amdgcn_raw_buffer_load_b128(vr, (uint32_t)(lane * 16), 1024 * k, kNT);
    sm.brow[lane] = br0 - b0;
    sm.brow[lane + 64] = br1 - b0;
#pragma unroll
    for (int k = 0; k < KQ; ++k) *reinterpret_cast<V4 *>(&sm.buf[(lane + 64 * k) * E]) = ch[k];
    if (q_tail < nq) {
        if (lane < E) {
            const int64_t g = abase + (int64_t)q_tail * E + lane;
            if (g < a.nnz) sm.buf[q_tail * E + lane] = vals[g];
        }
    }
    wave_sync();

    // 2. per word: this lane's value and X row offset (lane = mask bit). A
    // lane whose bit is clear keeps value 0 and an out-of-range offset (its
    // gathers return 0), so its products are +0 and the masks are not needed
    // after this pass.
    T v[NWM];
    uint32_t xo[NWM];
    const int slot = lane / Sh::RC;
    const int kcol = (lane % Sh::RC) % Sh::C;
    const uint32_t xrow = (uint32_t)a.ldx * (uint32_t)sizeof(T);
    {
        const uint64_t *__restrict__ gp = a.mw + w0;  // readable 512 bytes past the last word
        uint32_t vslot = (uint32_t)shift;
#pragma unroll
        for (int j = 0; j < NWM; ++j) {
            uint64_t m = nw > 0 ? gp[j] : 0ull;
            if (j == 0) m &= lo_mask;
            m = j < nw ? m : 0ull;
            const uint32_t s = lane_rank(m) + vslot;
            // lanes past the tile's values (bits of the next tile's blocks in
            // the last word) may read past the buffer: clamped, never used
            v[j] = pick(m, sm.buf[s < (uint32_t)SM::NBUF ? s : 0u], T(0));
            // the column of slot j BPW + slot: register (j BPW) / 64 of lane (j BPW + slot) mod 64
            const int c = __builtin_amdgcn_ds_bpermute(((j * Sh::BPW) % 64 + slot) * 4, colr[(j * Sh::BPW) / 64]);
            xo[j] = pick(m, (uint32_t)(c + kcol) * xrow, 0xffffffffu);
            vslot += (uint32_t)__popcll(m);
        }
    }
    // row-sum layout, fixed for all columns: L lanes per (interval, block
    // row); with more than 64 pairs (up to 128), L = 1 and a lane takes pairs
    // lane and lane + 64
    const int npairs = nI * Sh::R;
    const int lg = npairs > 64 ? 0 : npairs > 1 ? __builtin_clz((unsigned)(npairs - 1)) - 26 : 6;
    const int L = 1 << lg;
    const int l = lane & (L - 1);
    const int rounds = npairs > 64 ? 2 : 1;
    T *__restrict__ Y = static_cast<T *>(a.Y);
    // whether each row holds an entry (accumulate leaves empty rows alone)
    bool stored[2] = {false, false};
#pragma unroll
    for (int rd = 0; rd < 2; ++rd) {
        const int pair = (lane >> lg) + 64 * rd;
        if (rd < rounds && pair < npairs) {
            const int li = pair / Sh::R, rho = pair % Sh::R;
            const int bs = sm.brow[li], be = sm.brow[li + 1];
            if (Sh::R == 1) {
                stored[rd] = be > bs;
            } else if (a.accumulate) {
                for (int b = bs + l; b < be; b += L) {
                    const unsigned g = (unsigned)(b + lo_slot);
                    const uint32_t m = (uint32_t)(a.mw[w0 + g / Sh::BPW] >> ((g % Sh::BPW) * Sh::RC));
                    stored[rd] = stored[rd] || ((m >> (rho * Sh::C)) & Sh::CMASK) != 0;
                }
            }
        }
        if (Sh::R > 1 && a.accumulate)
            for (int m = L >> 1; m >= 1; m >>= 1) stored[rd] = __shfl_xor((int)stored[rd], m, 64) || stored[rd];
    }
    // Per column group, the products of each word are added over each block
    // row's C lanes (DPP) and the lane at column 0 of the block row stores
    // the (block, block row) partial at entry j (64 / C) + lane / C, i.e.
    // slot j BPW + slot, block row rho (entries of the next tile's blocks in
    // the last word are never read). L lanes per (interval, block row) then
    // add its partials, in the same order for every column.
    //
    // Columns are taken in groups of G = 16 / sizeof(T) when the launch says
    // every group is one aligned 16-byte piece of each X and Y row (a.wide):
    // one 128-bit gather per lane and word brings the group's G values, an
    // entry holds the group's G partials (16 bytes), the row sums read them
    // with wide loads and each row's G results are stored at once. Otherwise
    // the columns are taken one by one, one partial per entry. Both give the
    // same bits for a column.
    constexpr int G = 16 / (int)sizeof(T);
    // FP64 stops the lane sums at PPR = 2 partials per (block, block row)
    // (each 64-bit DPP step is two moves and an add); FP32 adds all C lanes
    constexpr int PPR = SM::PPR;
    constexpr int W = Sh::C / PPR;     // lanes added into one partial
    constexpr int PW = 64 / Sh::C * PPR;   // partial entries per word
    static_assert(SM::NWMAX * PW * G <= SM::NALL, "the partials must fit the buffer");
    const int pe = lane / W;           // this lane's partial entry within a word
    const bool keeper = kcol % W == 0; // the lanes that store their block row's partials
    auto lane_sum = [](T p) {
        if constexpr (sizeof(T) == 8) {
            p += dpp_f64<0xb1>(p);                          // quad_perm [1,0,3,2]
            if constexpr (W == 4) p += dpp_f64<0x4e>(p);    // quad_perm [2,3,0,1]
            return p;
        } else {
            return row_group_sum<Sh::C>(p);
        }
    };
    if (a.wide) {
        for (int q0 = 0; q0 < a.k; q0 += G) {
            const uint32_t qb = (uint32_t)q0 * (uint32_t)sizeof(T);
            V4 xw[NWM];
#pragma unroll
            for (int j = 0; j < NWM; ++j)
                xw[j] = __builtin_amdgcn_raw_buffer_load_b128(xr, xo[j] == 0xffffffffu ? 0xffffffffu : xo[j] + qb,
                                                              0, 0);
            wave_sync();  // the values (first group) or the previous group's sums are read
#pragma unroll
            for (int j = 0; j < NWM; ++j) {
                const T *xg = reinterpret_cast<const T *>(&xw[j]);
                T pg[G];
#pragma unroll
                for (int g = 0; g < G; ++g) pg[g] = lane_sum(v[j] * xg[g]);
                if (keeper) *reinterpret_cast<V4 *>(&sm.buf[(j * PW + pe) * G]) = *reinterpret_cast<const V4 *>(pg);
            }
            wave_sync();
#pragma unroll
            for (int rd = 0; rd < 2; ++rd) {
                const int pair = (lane >> lg) + 64 * rd;
                if (rd >= rounds) break;
                double acc[G], a1[G];
#pragma unroll
                for (int g = 0; g < G; ++g) acc[g] = a1[g] = 0.0;
                if (pair < npairs) {
                    const int li = pair / Sh::R, rho = pair % Sh::R;
                    const int bs = sm.brow[li], be = sm.brow[li + 1];
                    int b = bs + l;
                    for (; b + L < be; b += 2 * L) {
#pragma unroll
                        for (int h = 0; h < PPR; ++h) {
                            const V4 w0v = *reinterpret_cast<const V4 *>(
                                &sm.buf[(((b + lo_slot) * Sh::R + rho) * PPR + h) * G]);
                            const V4 w1v = *reinterpret_cast<const V4 *>(
                                &sm.buf[(((b + L + lo_slot) * Sh::R + rho) * PPR + h) * G]);
                            const T *e0 = reinterpret_cast<const T *>(&w0v);
                            const T *e1 = reinterpret_cast<const T *>(&w1v);
#pragma unroll
                            for (int g = 0; g < G; ++g) {
                                acc[g] += (double)e0[g];
                                a1[g] += (double)e1[g];
                            }
                        }
                    }
                    if (b < be) {
#pragma unroll
                        for (int h = 0; h < PPR; ++h) {
                            const V4 w0v = *reinterpret_cast<const V4 *>(
                                &sm.buf[(((b + lo_slot) * Sh::R + rho) * PPR + h) * G]);
                            const T *e0 = reinterpret_cast<const T *>(&w0v);
#pragma unroll
                            for (int g = 0; g < G; ++g) acc[g] += (double)e0[g];
                        }
                    }
#pragma unroll
                    for (int g = 0; g < G; ++g) acc[g] += a1[g];
                }
#pragma unroll
                for (int g = 0; g < G; ++g) acc[g] = group_sum(acc[g], lg);
                if (pair < npairs && l == 0) {
                    const int li = pair / Sh::R, rho = pair % Sh::R;
                    const int64_t row = (int64_t)(d.i0 + li) * Sh::R + rho;
                    if (row < a.n_rows) {
                        T *yp = Y + row * a.ldy + q0;
                        T out[G];
                        if (a.accumulate) {
                            const V4 old = *reinterpret_cast<const V4 *>(yp);
                            const T *o = reinterpret_cast<const T *>(&old);
#pragma unroll
                            for (int g = 0; g < G; ++g) out[g] = stored[rd] ? (T)(acc[g] + (double)o[g]) : o[g];
                        } else {
#pragma unroll
                            for (int g = 0; g < G; ++g) out[g] = (T)acc[g];
                        }
                        *reinterpret_cast<V4 *>(yp) = *reinterpret_cast<const V4 *>(out);
                    }
                }
            }
        }
        return;
    }
    for (int q = 0; q < a.k; ++q) {
        // gathers of column q for all words, then its partials
        T xv[NWM];
        const uint32_t qb = (uint32_t)q * (uint32_t)sizeof(T);
#pragma unroll
        for (int j = 0; j < NWM; ++j) xv[j] = buf_load<T>(xr, xo[j] == 0xffffffffu ? 0xffffffffu : xo[j] + qb);
        wave_sync();  // the values (first column) or the previous column's sums are read
#pragma unroll
        for (int j = 0; j < NWM; ++j) {
            const T p = lane_sum(v[j] * xv[j]);
            if (keeper) sm.buf[j * PW + pe] = p;
        }
        wave_sync();

        // row sums: L lanes per (interval, block row)
        const T *__restrict__ pu = sm.buf;
#pragma unroll
        for (int rd = 0; rd < 2; ++rd) {
            const int pair = (lane >> lg) + 64 * rd;
            if (rd >= rounds) break;
            double acc = 0.0;
            if (pair < npairs) {
                const int li = pair / Sh::R, rho = pair % Sh::R;
                const int bs = sm.brow[li], be = sm.brow[li + 1];
                double a0 = 0.0, a1 = 0.0;
                int b = bs + l;
                for (; b + L < be; b += 2 * L) {
#pragma unroll
                    for (int h = 0; h < PPR; ++h) {
                        a0 += (double)pu[((b + lo_slot) * Sh::R + rho) * PPR + h];
                        a1 += (double)pu[((b + L + lo_slot) * Sh::R + rho) * PPR + h];
                    }
                }
                if (b < be) {
#pragma unroll
                    for (int h = 0; h < PPR; ++h) a0 += (double)pu[((b + lo_slot) * Sh::R + rho) * PPR + h];
                }
                acc = a0 + a1;
            }
            acc = group_sum(acc, lg);
            if (pair < npairs && l == 0) {
                const int li = pair / Sh::R, rho = pair % Sh::R;
                const int64_t row = (int64_t)(d.i0 + li) * Sh::R + rho;
                if (row < a.n_rows) {
                    T *yp = Y + row * a.ldy + q;
                    if (a.accumulate) {
                        if (stored[rd]) *yp = (T)(acc + (double)*yp);
                    } else {
                        *yp = (T)acc;
                    }
                }
            }
        }
    }
}

template <class T>
__device__ __forceinline__ double ld_x(__amdgpu_buffer_rsrc_t xr, uint32_t off) {
    return (double)buf_load<T>(xr, off);
}

// One interval longer than a tile: lane = mask bit, k running sums per lane.
template <class Sh, class T>
__device__ void spmm_long(const SpmmArgs &a, const TileDesc &d, __amdgpu_buffer_rsrc_t xr) {
    const int lane = threadIdx.x & 63;
    const T *__restrict__ vals = static_cast<const T *>(a.vals);
    const int slot = lane / Sh::RC;
    const int kcol = (lane % Sh::RC) % Sh::C;
    const int b0 = d.b0, b1 = d.b1;
    const int w0 = b0 / Sh::BPW;
    const int nwt = (b1 - 1) / Sh::BPW - w0 + 1;
    const int lo_slot = b0 - w0 * Sh::BPW;
    const int end_bit = (b1 - w0 * Sh::BPW) * Sh::RC;
    const uint32_t xrow = (uint32_t)a.ldx * (uint32_t)sizeof(T);
    double acc[kMaxK];
#pragma unroll
    for (int q = 0; q < kMaxK; ++q) acc[q] = 0.0;
    int n_here = 0;
    int64_t vrun = d.vbase;
    for (int i = 0; i < nwt; ++i) {
        uint64_t m = a.mw[w0 + i];
        if (i == 0) m &= ~low_bits(lo_slot * Sh::RC);
        m &= low_bits(end_bit - 64 * i);
        if (__builtin_amdgcn_inverse_ballot_w64(m)) {
            const double v = (double)vals[vrun + lane_rank(m)];
            const uint32_t xo = (uint32_t)(a.bcol[(int64_t)(w0 + i) * Sh::BPW + slot] + kcol) * xrow;
            ++n_here;
#pragma unroll
            for (int q = 0; q < kMaxK; ++q)
                if (q < a.k) acc[q] = __builtin_fma(v, ld_x<T>(xr, xo + (uint32_t)(q * sizeof(T))), acc[q]);
        }
        vrun += __popcll(m);
    }
    // lanes of one block row: same (lane % RC) / C; add over column and slot bits
#pragma unroll
    for (int mm = 1; mm < Sh::C; mm <<= 1) {
        n_here += __shfl_xor(n_here, mm, 64);
#pragma unroll
        for (int q = 0; q < kMaxK; ++q) acc[q] += __shfl_xor(acc[q], mm, 64);
    }
#pragma unroll
    for (int mm = Sh::RC; mm < 64; mm <<= 1) {
        n_here += __shfl_xor(n_here, mm, 64);
#pragma unroll
        for (int q = 0; q < kMaxK; ++q) acc[q] += __shfl_xor(acc[q], mm, 64);
    }
    if (lane < Sh::RC && (lane % Sh::C) == 0) {
        const int64_t row = (int64_t)d.i0 * Sh::R + lane / Sh::C;
        if (row < a.n_rows) {
            T *__restrict__ Y = static_cast<T *>(a.Y) + row * a.ldy;
#pragma unroll
            for (int q = 0; q < kMaxK; ++q) {
                if (q < a.k) {
                    if (a.accumulate) {
                        if (n_here > 0) Y[q] = (T)(acc[q] + (double)Y[q]);
                    } else {
                        Y[q] = (T)acc[q];
                    }
                }
            }
        }
    }
}

// LDS of the row path (per wavefront).
template <class Sh, class T, int KQ>
struct RowsSmem {
    static constexpr int E = 16 / sizeof(T);
    static constexpr int WB = (64 * KQ - 1) * E;      // values a tile may hold
    static constexpr int NB = WB / Sh::RC;            // blocks a tile may hold
    static constexpr int NWMAX = NB / Sh::BPW + 2;
    static constexpr int NCR = (NWMAX * Sh::BPW + 63) / 64;
    static constexpr int NBR = (NB + 63) / 64;        // 64-lane rounds over the blocks
    int brow[128];                 // tile-relative interval pointers
    int pre[(NB + 1) * Sh::R];     // [block][block row]: that row's values in the tile's earlier blocks
    int rb[NB * Sh::R];            // [block][block row]: sorted place of the block row's first value
    int col[WB];                   // columns, sorted by row (and by column within a row)
    T val[WB];                     // values, in the same order
};

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v = max(v, __shfl_xor(v, m, 64));
    return v;
}

// One tile on the row path, all k columns (a.wide: k is a multiple of G).
template <class Sh, class T, int KQ>
__device__ void spmm_rows_tile(const SpmmArgs &a, const TileDesc &d, __amdgpu_buffer_rsrc_t xr,
                               RowsSmem<Sh, T, KQ> &sm) {
    using SM = RowsSmem<Sh, T, KQ>;
    using V4 = __attribute__((ext_vector_type(4))) unsigned int;
    constexpr int R = Sh::R, C = Sh::C, RC = Sh::RC, BPW = Sh::BPW;
    constexpr int NWM = SM::NWMAX;
    constexpr int G = 16 / (int)sizeof(T);
    const int lane = threadIdx.x & 63;
    const int b0 = d.b0, b1 = d.b1, nI = d.i1 - d.i0;
    const int nb = b1 - b0;
    const int w0 = b0 / BPW;
    const int nw = (b1 > b0) ? ((b1 - 1) / BPW - w0 + 1) : 0;
    const int lo_slot = b0 - w0 * BPW;
    const int end_bit = (b1 - w0 * BPW) * RC;   // bits of the tile's blocks end here (from word w0)
    const int cs0 = w0 * BPW;
    const int ncs = (int)(min<int64_t>((int64_t)(w0 + nw) * BPW, a.n_blocks) - cs0);

    // streams: block columns (slot lane + 64 k) and interval pointers
    const auto cr = rsrc(a.bcol + cs0, (uint32_t)(ncs > 0 ? ncs : 0) * 4u);
    int colr[SM::NCR];
#pragma unroll
    for (int k = 0; k < SM::NCR; ++k)
        colr[k] = __builtin_amdgcn_raw_buffer_load_b32(cr, (uint32_t)(lane * 4), 256 * k, kNT);
    const auto brr = rsrc(a.brow + d.i0, (uint32_t)(nI + 1) * 4u);
    const int br0 = __builtin_amdgcn_raw_buffer_load_b32(brr, (uint32_t)(lane * 4), 0, 0);
    const int br1 = __builtin_amdgcn_raw_buffer_load_b32(brr, (uint32_t)(lane * 4), 256, 0);
    // the tile's mask words and values: lane = mask bit, word j
    const uint64_t *__restrict__ gp = a.mw + w0;   // readable 512 bytes past the last word
    uint64_t mj[NWM];
#pragma unroll
    for (int j = 0; j < NWM; ++j) {
        uint64_t m = j < nw ? gp[j] : 0ull;
        if (j == 0) m &= ~low_bits(lo_slot * RC);
        mj[j] = m & low_bits(end_bit - 64 * j);
    }
    const auto vr = rsrc(static_cast<const T *>(a.vals) + d.vbase, (uint32_t)d.nv * (uint32_t)sizeof(T));
    T v[NWM];
    {
        uint32_t vslot = 0;
#pragma unroll
        for (int j = 0; j < NWM; ++j) {
            const uint64_t m = mj[j];
            v[j] = buf_load<T>(vr, pick(m, (vslot + lane_rank(m)) * (uint32_t)sizeof(T), 0xffffffffu));
            vslot += (uint32_t)__popcll(m);
        }
    }
    sm.brow[lane] = br0 - b0;
    sm.brow[lane + 64] = br1 - b0;

    // 1. lane = tile block: value counts of each block row, prefix over the tile
    int carry[R];
#pragma unroll
    for (int rho = 0; rho < R; ++rho) carry[rho] = 0;
#pragma unroll
    for (int k = 0; k < SM::NBR; ++k) {
        const int tb = lane + 64 * k;
        uint32_t mk = 0;
        if (tb < nb) {
            const int gs = tb + lo_slot;
            mk = (uint32_t)(gp[gs / BPW] >> ((gs % BPW) * RC)) & Sh::RCMASK;
        }
#pragma unroll
        for (int rho = 0; rho < R; ++rho) {
            const int c = __popc((mk >> (rho * C)) & Sh::CMASK);
            const int incl = wave_scan_dpp(c);
            if (tb < nb) sm.pre[tb * R + rho] = carry[rho] + incl - c;
            carry[rho] += __builtin_amdgcn_readlane(incl, 63);
        }
    }
#pragma unroll
    for (int rho = 0; rho < R; ++rho)
        if (lane == rho) sm.pre[nb * R + rho] = carry[rho];
    wave_sync();

    // 2. lane = interval: the sorted place of each block row's first value.
    // Rows are in order (interval, block row); within a row, the values in
    // block order, so in column order.
    for (int li = lane; li < nI; li += 64) {
        const int s0 = sm.brow[li], e0 = sm.brow[li + 1];
        int before = 0;
#pragma unroll
        for (int rho = 0; rho < R; ++rho) before += sm.pre[s0 * R + rho];
        int rs[R];
#pragma unroll
        for (int rho = 0; rho < R; ++rho) {
            rs[rho] = before - sm.pre[s0 * R + rho];
            before += sm.pre[e0 * R + rho] - sm.pre[s0 * R + rho];
        }
        for (int tb = s0; tb < e0; ++tb) {
#pragma unroll
            for (int rho = 0; rho < R; ++rho) sm.rb[tb * R + rho] = rs[rho] + sm.pre[tb * R + rho];
        }
    }
    wave_sync();

    // 3. lane = mask bit: each value and its column to their sorted place
    {
        const int slot = lane / RC;
        const int rho = (lane % RC) / C;
        const int kc = (lane % RC) % C;
        const uint64_t below_row = low_bits(slot * RC + rho * C);   // bits before this block row
#pragma unroll
        for (int j = 0; j < NWM; ++j) {
            const uint64_t m = mj[j];
            const int c = __builtin_amdgcn_ds_bpermute(((j * BPW) % 64 + slot) * 4, colr[(j * BPW) / 64]);
            if ((m >> lane) & 1ull) {
                const int tb = j * BPW + slot - lo_slot;
                const int rank = (int)lane_rank(m) - __popcll(m & below_row);
                const int pos = sm.rb[tb * R + rho] + rank;
                sm.val[pos] = v[j];
                sm.col[pos] = c + kc;
            }
        }
    }
    wave_sync();

    // 4. Q lanes per row: lane g of a row sums column group g (G columns)
    const int lgq = a.lgq;
    const int Q = 1 << lgq;
    const int g = lane & (Q - 1);
    const bool gon = g * G < a.k;
    const uint32_t xrow = (uint32_t)a.ldx * (uint32_t)sizeof(T);
    const uint32_t goff = (uint32_t)(g * 16);
    const int nrows = nI * R;
    T *__restrict__ Y = static_cast<T *>(a.Y);
    constexpr int U = 8;   // gathers in flight per lane
    for (int p0 = 0; p0 < nrows; p0 += (64 >> lgq)) {
        const int p = p0 + (lane >> lgq);
        int start = 0, len = 0;
        if (p < nrows) {
            const int li = p / R, rho = p % R;
            const int s0 = sm.brow[li], e0 = sm.brow[li + 1];
            len = sm.pre[e0 * R + rho] - sm.pre[s0 * R + rho];
            start = len > 0 ? sm.rb[s0 * R + rho] : 0;   // the row's first place (its first block's)
        }
        const int lmax = wave_max(len);
        double acc[G];
#pragma unroll
        for (int q = 0; q < G; ++q) acc[q] = 0.0;
        for (int u = 0; u < lmax; u += U) {
            V4 xw[U];
            T vv[U];
#pragma unroll
            for (int t = 0; t < U; ++t) {
                const bool ok = u + t < len;
                const int idx = ok ? start + u + t : 0;
                vv[t] = ok ? sm.val[idx] : T(0);
                const uint32_t off = (ok && gon) ? (uint32_t)sm.col[idx] * xrow + goff : 0xffffffffu;
                xw[t] = __builtin_amdgcn_raw_buffer_load_b128(xr, off, 0, 0);
            }
#pragma unroll
            for (int t = 0; t < U; ++t) {
                const T *xg = reinterpret_cast<const T *>(&xw[t]);
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    if constexpr (sizeof(T) == 8) acc[q] = __builtin_fma(vv[t], xg[q], acc[q]);
                    else acc[q] += (double)(vv[t] * xg[q]);
                }
            }
        }
        if (p < nrows && gon) {
            const int li = p / R, rho = p % R;
            const int64_t row = (int64_t)(d.i0 + li) * R + rho;
            if (row < a.n_rows && (len > 0 || !a.accumulate)) {
                T *yp = Y + row * a.ldy + g * G;
                T out[G];
                if (a.accumulate) {
                    const V4 old = *reinterpret_cast<const V4 *>(yp);
                    const T *o = reinterpret_cast<const T *>(&old);
#pragma unroll
                    for (int q = 0; q < G; ++q) out[q] = (T)(acc[q] + (double)o[q]);
                } else {
#pragma unroll
                    for (int q = 0; q < G; ++q) out[q] = (T)acc[q];
                }
                *reinterpret_cast<V4 *>(yp) = *reinterpret_cast<const V4 *>(out);
            }
        }
    }
}

template <int R, int C, class T, int KQ>
__global__ __launch_bounds__(kThreads) void k_spmm_rows(SpmmArgs a) {
    using Sh = Shape<R, C>;
    using SM = RowsSmem<Sh, T, KQ>;
    __shared__ SM sm[kWaves];
    int g = blockIdx.x;
    if (a.xcd_remap) g = (int)(blockIdx.x & 7u) * a.tiles_per_xcd + (int)(blockIdx.x >> 3);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = g * kWaves + wid;
    if (t >= a.n_tiles) return;
    const TileDesc d = a.tiles[t];
    const int64_t xbytes = a.n_cols > 0 ? ((a.n_cols - 1) * a.ldx + a.k) * (int64_t)sizeof(T) : 0;
    const auto xr = rsrc(a.X, (uint32_t)xbytes);
    if (d.b1 - d.b0 > SM::NB) spmm_long<Sh, T>(a, d, xr);
    else spmm_rows_tile<Sh, T, KQ>(a, d, xr, sm[wid]);
}

template <int R, int C, class T, int KQ>
__global__ __launch_bounds__(kThreads) void k_spmm_wave(SpmmArgs a) {
    using Sh = Shape<R, C>;
    using SM = SpmmSmem<Sh, T, KQ>;
    __shared__ SM sm[kWaves];
    int g = blockIdx.x;
    if (a.xcd_remap) g = (int)(blockIdx.x & 7u) * a.tiles_per_xcd + (int)(blockIdx.x >> 3);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = g * kWaves + wid;
    if (t >= a.n_tiles) return;
    const TileDesc d = a.tiles[t];
    // exactly the bytes of the k used columns: rows 0..n_cols-1, leading dimension ldx
    const int64_t xbytes = a.n_cols > 0 ? ((a.n_cols - 1) * a.ldx + a.k) * (int64_t)sizeof(T) : 0;
    const auto xr = rsrc(a.X, (uint32_t)xbytes);
    if (d.b1 - d.b0 > SM::NB) spmm_long<Sh, T>(a, d, xr);
    else spmm_tile<Sh, T, KQ>(a, d, xr, sm[wid]);
}

template <int R, int C, class T>
spc_status launch_rows(int kq, int cu_groups, dim3 grid, const SpmmArgs &a, hipStream_t s) {
    switch (kq) {
    case 2: return launch_capped(k_spmm_rows<R, C, T, 2>, cu_groups, grid, dim3(kThreads), s, a);
    case 6: return launch_capped(k_spmm_rows<R, C, T, 6>, cu_groups, grid, dim3(kThreads), s, a);
    case 8: return launch_capped(k_spmm_rows<R, C, T, 8>, cu_groups, grid, dim3(kThreads), s, a);
    default: return launch_capped(k_spmm_rows<R, C, T, 4>, cu_groups, grid, dim3(kThreads), s, a);
    }
}

template <int R, int C, class T>
spc_status launch(int kq, int cu_groups, dim3 grid, const SpmmArgs &a, hipStream_t s) {
    switch (kq) {
    case 2: return launch_capped(k_spmm_wave<R, C, T, 2>, cu_groups, grid, dim3(kThreads), s, a);
    case 6: return launch_capped(k_spmm_wave<R, C, T, 6>, cu_groups, grid, dim3(kThreads), s, a);
    case 8: return launch_capped(k_spmm_wave<R, C, T, 8>, cu_groups, grid, dim3(kThreads), s, a);
    default: return launch_capped(k_spmm_wave<R, C, T, 4>, cu_groups, grid, dim3(kThreads), s, a);
    }
}

}  // namespace

spc_status spmv_launch(const spc_beta_view *A, const spc_plan *P, const void *x, void *y, int accumulate,
                       hipStream_t stream);

spc_status spmm_launch(const spc_beta_view *A, const spc_plan *P, int k, const void *X, int64_t ldx, void *Y,
                       int64_t ldy, int accumulate, hipStream_t stream) {
    SpmmArgs a;
    a.brow = A->block_rowptr;
    a.bcol = A->block_colidx;
    a.mw = static_cast<const uint64_t *>(A->block_masks);
    a.vals = A->values;
    a.X = X;
    a.Y = Y;
    a.tiles = P->d_tiles;
    a.n_rows = A->n_rows;
    a.n_cols = A->n_cols;
    a.nnz = A->nnz;
    a.n_blocks = A->n_blocks;
    a.ldx = ldx;
    a.ldy = ldy;
    a.k = k;
    {
        // groups of G columns are whole aligned 16-byte pieces of every X row
        const int64_t es = A->dtype == SPC_F64 ? 8 : 4, G = 16 / es;
        // groups of G columns are whole aligned 16-byte pieces of every X and Y row
        a.wide = (k % G == 0) && ((ldx * es) % 16 == 0) && (reinterpret_cast<uintptr_t>(X) % 16 == 0) &&
                 ((ldy * es) % 16 == 0) && (reinterpret_cast<uintptr_t>(Y) % 16 == 0);
    }
    a.n_tiles = (int32_t)P->n_tiles;
    a.accumulate = accumulate;
    a.xcd_remap = P->xcd_remap;
    const int64_t groups = div_up(P->n_tiles, kWaves);
    a.tiles_per_xcd = (int32_t)div_up(groups, 8);
    dim3 grid(P->xcd_remap ? (unsigned)(8 * a.tiles_per_xcd) : (unsigned)groups);
    // the row path: lanes per row Q = the 16-byte groups of a row, rounded up to a power of two
    const int64_t es = A->dtype == SPC_F64 ? 8 : 4;
    const int64_t row_bytes = (int64_t)k * es;
    SPC_REQUIRE(P->spmm_path != SPC_SPMM_ROWS || a.wide, SPC_ERR_INVALID_ARG,
                "the row path needs k a multiple of %d and 16-byte aligned X and Y rows", (int)(16 / es));
    const bool rows = a.wide && (P->spmm_path == SPC_SPMM_ROWS || (P->spmm_path == SPC_SPMM_AUTO && row_bytes >= 64));
    a.lgq = 0;
    while ((16 << a.lgq) < row_bytes) ++a.lgq;
    return with_shape(P->shape, [&](auto sh) {
        using Sh = decltype(sh);
        return with_dtype(A->dtype, [&](auto tv) {
            using T = decltype(tv);
            if (rows) return launch_rows<Sh::R, Sh::C, T>(P->kq, P->cu_groups, grid, a, stream);
            return launch<Sh::R, Sh::C, T>(P->kq, P->cu_groups, grid, a, stream);
        });
    });
}

}  // namespace spc

extern "C" spc_status spc_spmm_beta(const spc_beta_view *A, const spc_plan *plan, int32_t k, const void *X,
                                    int64_t ldx, void *Y, int64_t ldy, int32_t accumulate, hipStream_t stream) {
    spc_status st = spc::check_view(A);
    if (st != SPC_OK) return st;
    spc::TempPlan tp(stream);
    if (plan == nullptr) {
        // one-off product: a default plan (mode 0) that lives for this call only
        if ((st = spc_plan_create(A, nullptr, &tp.p, stream)) != SPC_OK) return st;
        plan = tp.p;
    }
    SPC_REQUIRE(plan->mode == 0, SPC_ERR_INVALID_ARG, "spc_spmm_beta needs a plan of mode 0 (wavefront tiles)");
    SPC_REQUIRE(plan->A.block_rowptr == A->block_rowptr && plan->A.values == A->values &&
                    plan->A.block_masks == A->block_masks && plan->A.n_rows == A->n_rows,
                SPC_ERR_INVALID_ARG, "plan was built for a different matrix view");
    SPC_REQUIRE(k >= 1 && k <= spc::kMaxK, SPC_ERR_CAPACITY, "k must be in 1..%d", spc::kMaxK);
    SPC_REQUIRE(ldx >= k && ldy >= k, SPC_ERR_INVALID_ARG, "leading dimensions must be at least k");
    SPC_REQUIRE(accumulate == 0 || accumulate == 1, SPC_ERR_INVALID_ARG, "accumulate must be 0 or 1");
    if (A->n_rows == 0 || plan->n_tiles == 0) return SPC_OK;
    SPC_REQUIRE(X && Y, SPC_ERR_INVALID_ARG, "null X or Y");
    const size_t es = A->dtype == SPC_F64 ? 8 : 4;
    SPC_REQUIRE((uint64_t)A->n_cols * (uint64_t)ldx * es < 0xf0000000ull, SPC_ERR_CAPACITY,
                "X must be smaller than 3.75 GiB (32-bit offsets)");
    SPC_REQUIRE((reinterpret_cast<uintptr_t>(A->values) & 15u) == 0, SPC_ERR_INVALID_ARG,
                "spc_spmm_beta needs a 16-byte aligned values array");
    SPC_REQUIRE(reinterpret_cast<uintptr_t>(X) % es == 0 && reinterpret_cast<uintptr_t>(Y) % es == 0,
                SPC_ERR_INVALID_ARG, "X and Y must be aligned to the element size");
    // one contiguous right-hand side is a vector: the single-vector kernel
    if (k == 1 && ldx == 1 && ldy == 1) return spc::spmv_launch(A, plan, X, Y, accumulate, stream);
    return spc::spmm_launch(A, plan, k, X, ldx, Y, ldy, accumulate, stream);
}
