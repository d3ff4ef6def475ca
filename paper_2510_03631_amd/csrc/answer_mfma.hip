// Batched Answer and offline hint on the int8 matrix cores.
//
//   Out[r][b] = sum_j D[r][j] * Q[j][b]   mod 2^32   (LWE form)
//   Out[r][b] = sum_j D[r][j] * Q[j][b]   mod p      (field form, p < 2^32)
//
// The LWE form is the multi-request response of Section 5.2 (Algorithm 4's
// batched product, here over Z/2^32); the hint H = D A is the same product
// with A in place of Q (Section 5.3's offline work).  The field form is the
// server product of the Goldberg / FTR instantiation (Section 5.1), the
// "mod q" of Algorithm 4.
//
// gfx950 has only signed int8 matrix instructions, so both operands are
// centred.  With q = sum_k 2^(8k) q_k (byte limbs), q_k = q'_k + 128 and
// D = D' + 128 (D' = D xor 0x80 read as int8, likewise q'_k), over the
// integers:
//
//   D q = sum_k 2^(8k) (D' q'_k)  +  128 (colsum(q) - C * 0x80808080)
//                                 +  0x80808080 rowsum(D)
//
// One int8 GEMM with M = R, K = C and N = 4 * B (the four limb planes of
// every query side by side) gives the products P_k = D' q'_k; the epilogue
// adds P_0 + 2^8 P_1 + 2^16 P_2 + 2^24 P_3 and the two terms (column sums
// from the ingest kernel, row sums from the database handle).
// * Modulo 2^32 the int32 accumulators wrap freely: only residues are used.
// * The field form rebuilds D q exactly, modulo 2^64 (D q < 2^64 for
//   C <= 2^23), and reduces it mod p.  A product P_k over K <= 2^17 columns
//   lies in [-16256 K, 16384 K]: the int32 accumulator holds it exactly
//   except for +2^31 (all products (-128)(-128) with K = 2^17), which reads
//   back as -2^31, a value the true sum cannot take, and is mapped back.  So
//   every accumulation in the field form covers at most 2^17 columns; longer
//   rows are split along K (below).
//
// Split-K.  When the output tiles cannot fill the chip (few rows: the
// incremental hint, short databases), or the field form needs it, the K
// range is cut into S pieces; each workgroup writes its piece's limb
// combination as a partial (4 bytes mod 2^32, or 8 bytes exact) and a
// finishing kernel adds the S partials and the centring terms.
//
// Kernels
//   k_zero_words  clear the column sums
//   k_ingest      Q -> QL (N x Cp centred int8, K-contiguous) and exact
//                 64-bit colsum[b] = sum_j Q[j][b]
//   k_gemm_ring   int8 MFMA 32x32x32; global tiles go straight to LDS
//                 (global_load_lds_dwordx4) into a ring of stages; fused
//                 epilogue, optional row gather, optional split-K
//   k_gemm_roles  the same with separate loader waves for D and QL
//   k_gemm        register-staged LDS tiles, for databases the ring cannot
//                 serve (unaligned rows or C not a multiple of 16)
//   k_finish      sums split-K partials and adds the centring terms
//
// QL row index of (query b, limb k): n = (b / 32) * 128 + k * 32 + (b % 32),
// so the four limbs of a query land in the same lane of four adjacent 32x32
// output tiles and the epilogue combines them in registers.  Batches of at
// most 16 queries may use the narrow layout n = (b / 8) * 32 + k * 8 + b % 8
// instead: one 32-column tile holds all four limbs of 8 queries, so a batch
// of 8 is not padded to 32 queries; the epilogue then combines the limbs
// of a query across lanes c, c+8, c+16, c+24 with two shuffles.  QL is stored in
// 4 KiB tiles of 32 rows x 128 bytes (tile (n/32, k/128) at
// ((n/32) * Cp/128 + k/128) * 4096, row n%32 at 128 (n%32) within it): the
// ingest writes whole tiles and a 1 KiB block of a GEMM k-tile is contiguous.
#include "qpir_internal.h"

namespace {

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;
typedef unsigned long long u64;

constexpr uint32_t kCentreWord = 0x80808080u;
constexpr int kCpolNT = 2;   // cache-policy operand of a load: nt (non-temporal) on gfx950
constexpr int kKPad = 256;                    // QL rows are zero-padded to a multiple of this
constexpr uint32_t kExactSpan = 1u << 17;     // columns one exact int32 accumulation may cover
constexpr uint32_t kMaxExactCols = 1u << 23;  // D q < 2^64 and exact row sums
constexpr uint32_t kMaxSplits = 16;           // split-K pieces chosen for occupancy


// Epilogue modes.
enum : int {
    kFinal32 = 0,     // Out mod 2^32
    kPart32 = 1,      // split partial sum_k 2^(8k) P_k mod 2^32 (no centring terms)
    kFinalModP = 2,   // Out mod p
    kPart64 = 3,      // split partial sum_k 2^(8k) P_k, exact (mod 2^64)
};

__global__ void k_zero_words(uint32_t* __restrict__ p, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Block: 128 query coordinates j x 64 queries b.  Element (j, b) of the
// query matrix is Q[j * ldj + b * ldb].  Loads are coalesced along b for the
// row-major layout (ldb == 1: a wave reads 64 consecutive words of one row)
// and along j for the query-major one (QMAJOR, ldj == 1).  The tile goes
// through LDS with rows padded to 129 words, so that the stores hit 64
// distinct banks.  The block's QL rows 4*b0 .. 4*b0+255 (either layout)
// are consecutive 128-byte runs of the tiled layout; in the write phase lane l of a wave
// packs and stores 16-byte chunk l % 8 of row l / 8, so one store covers
// eight whole rows (1 KiB).  (Storing a thread's whole row as eight 16-byte
// pieces made every store touch 64 lines: 1.6 TB/s at 128 queries.)  The
// rows of limb 0 also sum their words: three lane shuffles combine the
// eight chunks of a row, and one lane adds the exact column sum.
constexpr int kIngJ = 128;
constexpr int kIngB = 64;

// VEC: 16-byte loads (4 consecutive queries of a row, or 4 consecutive
// coordinates of a query), when the query matrix is 16-byte aligned and the
// contiguous extent (B, or C for QMAJOR) is a multiple of 4; each thread then
// has its whole share of the tile (8 loads, 128 bytes) in flight at once.
template <bool QMAJOR, bool VEC>
__global__ __launch_bounds__(256) void k_ingest(const uint32_t* __restrict__ Q, uint64_t ldj,
                                                uint64_t ldb, uint32_t C, uint32_t B, uint32_t Bp,
                                                uint32_t Cp, int8_t* __restrict__ QL,
                                                u64* __restrict__ colsum, bool narrow) {
    __shared__ uint32_t s[kIngB][kIngJ + 1];
    const int t = threadIdx.x;
    // Query blocks vary fastest across the grid, so the blocks that read one
    // row of a row-major Q (64 queries each) are dispatched together.
    const uint32_t b0 = blockIdx.x * (uint32_t)kIngB;
    const uint32_t j0 = blockIdx.y * (uint32_t)kIngJ;
    if (VEC && QMAJOR) {
        const int j4 = t & 31, br = t >> 5;
        const uint32_t j = j0 + 4u * j4;
        u32x4 v[8];
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const uint32_t b = b0 + br + 8 * p;
            v[p] = (j < C && b < B)
                       ? *reinterpret_cast<const u32x4*>(Q + (uint64_t)b * ldb + j)
                       : u32x4{0, 0, 0, 0};
        }
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const int bl = br + 8 * p;
            s[bl][4 * j4 + 0] = v[p].x;
            s[bl][4 * j4 + 1] = v[p].y;
            s[bl][4 * j4 + 2] = v[p].z;
            s[bl][4 * j4 + 3] = v[p].w;
        }
    } else if (VEC) {
        const int q4 = t & 15, jr = t >> 4;
        const uint32_t b = b0 + 4u * q4;
        u32x4 v[8];
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const uint32_t j = j0 + jr + 16 * p;
            v[p] = (j < C && b < B)
                       ? *reinterpret_cast<const u32x4*>(Q + (uint64_t)j * ldj + b)
                       : u32x4{0, 0, 0, 0};
        }
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const int jl = jr + 16 * p;
            s[4 * q4 + 0][jl] = v[p].x;
            s[4 * q4 + 1][jl] = v[p].y;
            s[4 * q4 + 2][jl] = v[p].z;
            s[4 * q4 + 3][jl] = v[p].w;
        }
    } else if (QMAJOR) {
        const int jl = t & (kIngJ - 1);
        const uint32_t j = j0 + jl;
#pragma unroll 8
        for (int p = 0; p < kIngB / 2; ++p) {
            const int bl = (t >> 7) + 2 * p;
            const uint32_t b = b0 + bl;
            s[bl][jl] = (j < C && b < B) ? Q[(uint64_t)j * ldj + (uint64_t)b * ldb] : 0u;
        }
    } else {
        const int bl = t & (kIngB - 1);
        const uint32_t b = b0 + bl;
#pragma unroll 8
        for (int p = 0; p < kIngJ / 4; ++p) {
            const int jl = (t >> 6) + 4 * p;
            const uint32_t j = j0 + jl;
            s[bl][jl] = (j < C && b < B) ? Q[(uint64_t)j * ldj + (uint64_t)b * ldb] : 0u;
        }
    }
    __syncthreads();
    const int e = t & 7;                       // 16-byte chunk of the row
    const uint32_t n0 = 4u * b0;               // first QL row of the block, either layout
#pragma unroll 2
    for (int rnd = 0; rnd < 8; ++rnd) {
        const int R = rnd * 32 + (t >> 3);     // row of the block, 0..255
        // Wide: R = 128 g + 32 limb + b % 32; narrow: R = 32 g + 8 limb + b % 8.
        // Either way limb and the 8-query group of b are uniform per wave.
        const int limb = narrow ? (R & 31) >> 3 : (R & 127) >> 5;
        const int bl = narrow ? (R >> 5) * 8 + (R & 7) : (R >> 7) * 32 + (R & 31);
        const uint32_t b = b0 + bl;
        if (b >= Bp) continue;                 // uniform per wave (Bp % 8 == 0): no QL row
        const bool live = b < B;
        uint32_t w[4];
        u64 sum = 0;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            uint32_t word = 0;
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                const int jl = 16 * e + 4 * x + y;
                const uint32_t v = s[bl][jl];
                if (limb == 0) sum += v;
                const uint32_t byte =
                    (live && j0 + jl < C) ? (((v >> (8 * limb)) & 0xFFu) ^ 0x80u) : 0u;
                word |= byte << (8 * y);
            }
            w[x] = word;
        }
        *reinterpret_cast<u32x4*>(QL + ql_row(n0 + R, Cp) + ql_col(j0) + 16 * e) =
            u32x4{w[0], w[1], w[2], w[3]};
        if (limb == 0) {
            sum += __shfl_xor(sum, 1);
            sum += __shfl_xor(sum, 2);
            sum += __shfl_xor(sum, 4);
            if (e == 0 && live) atomicAdd(&colsum[b], sum);
        }
    }
}

// ---------------------------------------------------------------- epilogue
struct Epi {
    uint32_t M;                 // output rows (gathered rows, or R)
    uint32_t B, R, C;
    const uint32_t* rows;       // database row of output row i, or null
    const u64* colsum;          // exact column sums, B words
    const uint32_t* rowsum;     // exact row sums (handle metadata)
    uint32_t* out;
    uint64_t o_ldr, o_ldb;
    void* part;                 // split-K partials [split][M][B]
    uint32_t p;                 // modulus of the field form
};

__device__ inline uint32_t colterm32(const Epi& e, uint32_t b) {
    return 128u * ((uint32_t)e.colsum[b] - e.C * kCentreWord);
}

__device__ inline u64 colterm64(const Epi& e, uint32_t b) {
    return 128ull * (e.colsum[b] - (u64)e.C * kCentreWord);
}

// Exact value of a limb product read from its int32 accumulator (K <= 2^17).
__device__ inline u64 limb64(int32_t v) {
    return v == INT32_MIN ? (1ull << 31) : (u64)(int64_t)v;
}

// Output element (local row i, query b) from its limb combination
// x = sum_k 2^(8k) P_k (exact; only x mod 2^32 matters in the 32-bit modes).
template <int MODE, bool GATHER>
__device__ inline void epi_put(const Epi& e, uint32_t split, uint32_t i, uint32_t b, u64 x) {
    if (i >= e.M || b >= e.B) return;
    if (MODE == kFinal32 || MODE == kFinalModP) {
        const uint32_t r = GATHER ? e.rows[i] : i;
        if (r >= e.R) return;
        uint32_t* dst = e.out + (uint64_t)r * e.o_ldr + (uint64_t)b * e.o_ldb;
        if (MODE == kFinal32)
            *dst = (uint32_t)x + colterm32(e, b) + kCentreWord * e.rowsum[r];
        else
            *dst = (uint32_t)((x + colterm64(e, b) + (u64)kCentreWord * e.rowsum[r]) % e.p);
    } else {
        const uint64_t at = ((uint64_t)split * e.M + i) * e.B + b;
        if (MODE == kPart32)
            static_cast<uint32_t*>(e.part)[at] = (uint32_t)x;
        else
            static_cast<u64*>(e.part)[at] = x;
    }
}

// Limb combination of four limb products (wide layout).
template <int MODE, bool GATHER>
__device__ inline void epi_store(const Epi& e, uint32_t split, uint32_t i, uint32_t b, int32_t p0,
                                 int32_t p1, int32_t p2, int32_t p3) {
    if (MODE == kFinal32 || MODE == kPart32)
        epi_put<MODE, GATHER>(e, split, i, b,
                              (uint32_t)p0 + ((uint32_t)p1 << 8) + ((uint32_t)p2 << 16) +
                                  ((uint32_t)p3 << 24));
    else
        epi_put<MODE, GATHER>(e, split, i, b,
                              limb64(p0) + (limb64(p1) << 8) + (limb64(p2) << 16) +
                                  (limb64(p3) << 24));
}

// Write a wave's accumulators through the epilogue: the four limb tiles of
// query group g sit in acc[a][4g .. 4g+3] (C layout of the 32x32 MFMA: lane
// holds column lane % 32, register v holds row 8 (v/4) + 4 (lane/32) + v%4).
template <int MODE, bool GATHER, int TM, int TN>
__device__ inline void epi_wave(const Epi& e, uint32_t split, const i32x16 (&acc)[TM][TN],
                                uint32_t m_base, uint32_t n_base, int lane) {
#pragma unroll
    for (int g = 0; g < TN / 4; ++g) {
        const uint32_t bq = n_base / 4u + 32u * g + (uint32_t)(lane & 31);
#pragma unroll
        for (int a = 0; a < TM; ++a) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const uint32_t i = m_base + a * 32 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
                epi_store<MODE, GATHER>(e, split, i, bq, acc[a][4 * g][v], acc[a][4 * g + 1][v],
                                        acc[a][4 * g + 2][v], acc[a][4 * g + 3][v]);
            }
        }
    }
}

// Narrow layout: in 32-column tile t of a wave, lane column c holds limb
// c / 8 of query n_base / 4 + 8 t + c % 8 (C layout as above).  The four
// limbs of a query sit in lanes c, c ^ 8, c ^ 16, c ^ 24 of the same half
// wave; two xor shuffles add the shifted products and lanes with c < 8
// store.
template <int MODE, bool GATHER, int TM, int TN>
__device__ inline void epi_wave_narrow(const Epi& e, uint32_t split, const i32x16 (&acc)[TM][TN],
                                       uint32_t m_base, uint32_t n_base, int lane) {
    const int c = lane & 31;
    const int limb = c >> 3;
#pragma unroll
    for (int t = 0; t < TN; ++t) {
        const uint32_t bq = n_base / 4u + 8u * t + (uint32_t)(c & 7);
#pragma unroll
        for (int a = 0; a < TM; ++a) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const uint32_t i = m_base + a * 32 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
                u64 x;
                if (MODE == kFinal32 || MODE == kPart32) {
                    uint32_t y = (uint32_t)acc[a][t][v] << (8 * limb);
                    y += __shfl_xor(y, 8);
                    y += __shfl_xor(y, 16);
                    x = y;
                } else {
                    x = limb64(acc[a][t][v]) << (8 * limb);
                    x += __shfl_xor(x, 8);
                    x += __shfl_xor(x, 16);
                }
                if (limb == 0) epi_put<MODE, GATHER>(e, split, i, bq, x);
            }
        }
    }
}

// Sum of the split partials plus the centring terms, one output per thread.
template <bool EXACT>
__global__ __launch_bounds__(256) void k_finish(Epi e, uint32_t splits) {
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (uint64_t)e.M * e.B) return;
    const uint32_t i = (uint32_t)(idx / e.B), b = (uint32_t)(idx % e.B);
    const uint32_t r = e.rows ? e.rows[i] : i;
    if (r >= e.R) return;
    const uint64_t plane = (uint64_t)e.M * e.B;
    uint32_t* dst = e.out + (uint64_t)r * e.o_ldr + (uint64_t)b * e.o_ldb;
    if (EXACT) {
        u64 v = colterm64(e, b) + (u64)kCentreWord * e.rowsum[r];
        const u64* part = static_cast<const u64*>(e.part) + idx;
        for (uint32_t s = 0; s < splits; ++s) v += part[s * plane];
        *dst = (uint32_t)(v % e.p);
    } else {
        uint32_t v = colterm32(e, b) + kCentreWord * e.rowsum[r];
        const uint32_t* part = static_cast<const uint32_t*>(e.part) + idx;
        for (uint32_t s = 0; s < splits; ++s) v += part[s * plane];
        *dst = v;
    }
}

// The same for the mod 2^32 form, four queries per thread with 16-byte
// partial loads and output stores (B % 4 == 0, queries contiguous and the
// output rows 16-byte aligned): a quarter of the threads and address
// arithmetic for a pass that only streams the partials.
__global__ __launch_bounds__(256) void k_finish4(Epi e, uint32_t splits) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;   // group of 4 outputs
    const uint32_t B4 = e.B / 4u;
    if (g >= (uint64_t)e.M * B4) return;
    const uint32_t i = (uint32_t)(g / B4), b = 4u * (uint32_t)(g % B4);
    const uint32_t r = e.rows ? e.rows[i] : i;
    if (r >= e.R) return;
    const uint64_t plane4 = (uint64_t)e.M * B4;
    const uint32_t rs = kCentreWord * e.rowsum[r];
    u32x4 v = u32x4{colterm32(e, b) + rs, colterm32(e, b + 1) + rs, colterm32(e, b + 2) + rs,
                    colterm32(e, b + 3) + rs};
    const u32x4* part = static_cast<const u32x4*>(e.part) + g;
    for (uint32_t s = 0; s < splits; ++s) v += part[s * plane4];
    *reinterpret_cast<u32x4*>(e.out + (uint64_t)r * e.o_ldr + b) = v;
}

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
// contiguous range of workgroup indices, so the tiles it runs at once are
// neighbours (shared D rows and query tiles stay in its own L2).
__device__ inline uint32_t xcd_remap(uint32_t bid, uint32_t nblk) {
    const uint32_t per = nblk / 8u;
    return bid < per * 8u ? (bid % 8u) * per + bid / 8u : bid;
}

// Tile of a (remapped) workgroup index, split-major: within a split, tiles
// go in groups of `group` row tiles (8 over a whole database) so the ~32
// workgroups an XCD runs at once share D and QL tiles in its L2.  Gathered
// rows take every row tile of a column tile as one group: their few row
// tiles then read each limb-plane tile together.
struct TileId {
    uint32_t m, n, split;
};

__device__ inline TileId tile_of(uint32_t bid, uint32_t n_tiles, uint32_t m_tiles,
                                 uint32_t kGroup = 8) {
    const uint32_t tiles = n_tiles * m_tiles;
    TileId t;
    t.split = bid / tiles;
    bid %= tiles;
    const uint32_t first_m = (bid / (kGroup * n_tiles)) * kGroup;
    const uint32_t gsize = min(m_tiles - first_m, kGroup);
    const uint32_t in_group = bid % (kGroup * n_tiles);
    t.m = first_m + in_group % gsize;
    t.n = in_group / gsize;
    return t;
}

// ---------------------------------------------------------------- GEMM, register-staged
template <int WM_, int WN_, int TM_, int TN_, int BK_>
struct Tile {
    static constexpr int WM = WM_, WN = WN_, TM = TM_, TN = TN_, BK = BK_;
    static constexpr int BM = WM * TM * 32;
    static constexpr int BN = WN * TN * 32;
    static constexpr int LDK = BK + 16;              // padded LDS row, bytes
    static constexpr int A_LOADS = BM * BK / (256 * 16);
    static constexpr int B_LOADS = BN * BK / (256 * 16);
    static constexpr int SEGS = BK / 16;             // 16-byte pieces per row
    static_assert(WM * WN == 4, "four waves");
    static_assert(TN % 4 == 0, "a wave covers whole groups of four limbs");
    static_assert(A_LOADS >= 1 && B_LOADS >= 1, "tile too small for 256 threads");
};

template <bool VEC>
__device__ inline u32x4 load_row16(const uint8_t* row, uint32_t k, uint32_t C) {
    if (VEC && k + 16 <= C) return *reinterpret_cast<const u32x4*>(row + k);
    uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const uint32_t b = (k + e < C) ? row[k + e] : 0u;
        w[e >> 2] |= b << (8 * (e & 3));
    }
    return u32x4{w[0], w[1], w[2], w[3]};
}

// Block tile BM x BN of Out; 4 waves in a WM x WN grid, each computing
// (TM*32) x (TN*32) with 32x32x32 int8 MFMAs; LDS tiles staged through
// registers with one tile of prefetch.  LWE form, no split.
template <class T, bool VEC, bool GATHER>
__global__ __launch_bounds__(256) void k_gemm(const uint8_t* __restrict__ D, uint64_t pitch,
                                              const int8_t* __restrict__ QL, uint32_t Cp,
                                              uint32_t n_tiles, Epi e) {
    __shared__ __attribute__((aligned(16))) uint8_t sA[T::BM * T::LDK];
    __shared__ __attribute__((aligned(16))) uint8_t sB[T::BN * T::LDK];
    const uint32_t R = e.R, C = e.C, M = e.M;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / T::WN;
    const int wn = wave % T::WN;

    const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t m0 = (bid / n_tiles) * T::BM;
    const uint32_t n0 = (bid % n_tiles) * T::BN;

    // Global load assignment: thread -> (row, 16-byte segment).
    const int seg = tid % T::SEGS;
    const int rsub = tid / T::SEGS;
    constexpr int ROWS_PER_PASS = 256 / T::SEGS;

    const uint8_t* arow[T::A_LOADS];
#pragma unroll
    for (int p = 0; p < T::A_LOADS; ++p) {
        uint32_t i = m0 + rsub + p * ROWS_PER_PASS;
        i = i < M ? i : M - 1;
        const uint32_t r = GATHER ? e.rows[i] : i;
        arow[p] = D + (uint64_t)(r < R ? r : R - 1) * pitch;
    }
    const int8_t* brow[T::B_LOADS];
#pragma unroll
    for (int p = 0; p < T::B_LOADS; ++p)
        brow[p] = QL + ql_row(n0 + rsub + p * ROWS_PER_PASS, Cp);

    u32x4 ra[T::A_LOADS], rb[T::B_LOADS];
    auto gload = [&](uint32_t k0) {
        const uint32_t k = k0 + 16u * seg;
#pragma unroll
        for (int p = 0; p < T::A_LOADS; ++p) ra[p] = load_row16<VEC>(arow[p], k, C);
#pragma unroll
        for (int p = 0; p < T::B_LOADS; ++p)
            rb[p] = *reinterpret_cast<const u32x4*>(brow[p] + ql_col(k));
    };
    auto lstore = [&]() {
#pragma unroll
        for (int p = 0; p < T::A_LOADS; ++p) {
            const u32x4 v = ra[p] ^ u32x4{kCentreWord, kCentreWord, kCentreWord, kCentreWord};
            *reinterpret_cast<u32x4*>(&sA[(rsub + p * ROWS_PER_PASS) * T::LDK + 16 * seg]) = v;
        }
#pragma unroll
        for (int p = 0; p < T::B_LOADS; ++p)
            *reinterpret_cast<u32x4*>(&sB[(rsub + p * ROWS_PER_PASS) * T::LDK + 16 * seg]) = rb[p];
    };

    i32x16 acc[T::TM][T::TN];
#pragma unroll
    for (int a = 0; a < T::TM; ++a)
#pragma unroll
        for (int b = 0; b < T::TN; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[a][b][v] = 0;

    const int frag_row = lane & 31;
    const int frag_k = 16 * (lane >> 5);

    gload(0);
    lstore();
    __syncthreads();
    for (uint32_t k0 = 0; k0 < C; k0 += T::BK) {
        const bool more = k0 + T::BK < C;
        if (more) gload(k0 + T::BK);
#pragma unroll
        for (int ks = 0; ks < T::BK / 32; ++ks) {
            i32x4 fa[T::TM], fb[T::TN];
#pragma unroll
            for (int a = 0; a < T::TM; ++a)
                fa[a] = *reinterpret_cast<const i32x4*>(
                    &sA[(wm * T::TM * 32 + a * 32 + frag_row) * T::LDK + ks * 32 + frag_k]);
#pragma unroll
            for (int b = 0; b < T::TN; ++b)
                fb[b] = *reinterpret_cast<const i32x4*>(
                    &sB[(wn * T::TN * 32 + b * 32 + frag_row) * T::LDK + ks * 32 + frag_k]);
#pragma unroll
            for (int a = 0; a < T::TM; ++a)
#pragma unroll
                for (int b = 0; b < T::TN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
        if (more) {
            lstore();
            __syncthreads();
        }
    }
    epi_wave<kFinal32, GATHER, T::TM, T::TN>(e, 0, acc, m0 + wm * T::TM * 32,
                                              n0 + wn * T::TN * 32, lane);
}

// ---------------------------------------------------------------- LDS ring helpers
// 16-byte slot of (row, segment) in an LDS row.  A fragment read has 32
// lanes on 32 consecutive rows at one segment; gfx950's LDS serves a
// 16-byte read 16 lanes at a time across 64 four-byte banks, so the 16 rows
// of a pass must land on 16 distinct 16-byte bank groups.  A 64-byte row
// spans 16 banks (row % 4 picks the quarter of the bank space), a 128-byte
// row 32 banks (row % 2); XORing the segment with the next row bits fills
// the remaining choices.  (Measured: a swizzle that is conflict-free for
// 8 lanes over 32 banks spent half of the LDS cycles in bank conflicts.)
template <int BK>
__device__ inline int swz(int row, int seg) {
    return BK == 64 ? (seg ^ ((row >> 2) & 3)) : (seg ^ ((row >> 1) & 7));
}

// s_waitcnt with only vmcnt constrained (gfx9 encoding: vmcnt low bits
// [3:0], high bits [15:14]; expcnt and lgkmcnt left at their maximum).
template <int N>
__device__ inline void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// Workgroup barrier without the memory fence of __syncthreads(): the fence
// would drain every outstanding load (vmcnt(0)) and empty the ring.  Each
// wave has already waited for its own tile loads (wait_vmcnt), and LDS
// reads are not moved across the asm statements.
__device__ inline void ring_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// ---------------------------------------------------------------- GEMM, LDS ring
// The main kernel for aligned databases with C a multiple of 16.  Global
// tiles go straight to LDS with global_load_lds_dwordx4 (no register
// staging), into a ring of STAGES k-tiles of BK bytes, so STAGES-1 tiles are
// in flight while one is consumed.  Centring of D (xor 0x80) is applied to
// the A fragments in registers.
// DX_ > 0 gives D DX_ more ring slots than the limb planes (SA = STAGES +
// DX_ D tiles against SB = STAGES QL tiles), QX_ > 0 the limb planes QX_
// more than D: the deeper operand's tiles are issued that many stages
// earlier than the tiles of the other they meet.
template <int WM_, int WN_, int TM_, int TN_, int STAGES_, int BK_ = 64, bool NARROW_ = false,
          int DX_ = 0, int QX_ = 0>
struct Ring {
    static constexpr int WM = WM_, WN = WN_, TM = TM_, TN = TN_, STAGES = STAGES_;
    static constexpr int DX = DX_, QX = QX_;
    static constexpr int SA = STAGES + DX, SB = STAGES + QX;   // D and QL ring slots
    static constexpr int SMAX = SA > SB ? SA : SB;
    static_assert(DX == 0 || QX == 0, "one operand runs deeper");
    static constexpr bool NARROW = NARROW_;              // narrow QL layout (8 queries per tile)
    static constexpr int NW = WM * WN;                   // waves per workgroup
    static constexpr int THREADS = 64 * NW;
    static constexpr int BK = BK_;                       // k bytes per stage: 64 or 128
    static constexpr int SEGS = BK / 16;                 // 16-byte slots per LDS row
    static constexpr int RPB = 1024 / BK;                // rows per 1 KiB block
    static constexpr int BM = WM * TM * 32;
    static constexpr int BN = WN * TN * 32;
    static constexpr int A_BYTES = BM * BK;
    static constexpr int B_BYTES = BN * BK;
    static constexpr int STAGE_BYTES = (BM + BN) * BK;
    static constexpr int A_BLOCKS = BM / RPB;            // 1 KiB blocks
    static constexpr int BLOCKS = (BM + BN) / RPB;
    static constexpr int LOADS = BLOCKS / NW;            // per wave per tile
    static constexpr int LDS_BYTES = SA * A_BYTES + SB * B_BYTES;
    static_assert(BK == 64 || BK == 128, "64- or 128-byte stages");
    static_assert(NW == 4 || NW == 8, "four or eight waves");
    static_assert(NARROW || TN % 4 == 0, "a wave covers whole groups of four limbs");
    static_assert(BLOCKS % NW == 0, "blocks split evenly over waves");
    static_assert(A_BLOCKS % NW == 0, "a wave's first A_LOADS loads carry D rows");
    static constexpr int A_LOADS = A_BLOCKS / NW;
    static constexpr int B_LOADS = LOADS - A_LOADS;
    // Per stage a wave issues LOADS loads, one list: D first then QL (DX
    // == 0), or QL first then D (DX > 0): the deeper operand goes last, so
    // its tile issued after the other's may stay in flight while that one
    // is consumed.  Loads complete in order; at the start of stage u at most
    // QL_WAIT of this wave's loads may still be outstanding for tiles u (D
    // and QL) to have landed: the deeper operand's loads of the stage that
    // issued the other operand's tile u, plus the stages after it.
    static constexpr int QL_WAIT =
        (DX > 0 ? A_LOADS : 0) + (QX > 0 ? LOADS - A_LOADS : 0) + (STAGES - 2) * LOADS;
    // The loads of the tile that refills a freed slot are spread over all
    // KS k-steps of a stage when another tile is in flight (three or more
    // stages, or a D ring one tile deeper, whose D tile then has two stages
    // to land), else over the fewest k-steps that fit (one load per MFMA),
    // so the tile has the rest of the stage to land.  (Deeper D ring, 64
    // queries at 32768^2: 380-384 us with the loads in the first k-step,
    // 347-357 us spread; the two-stage ring and a deeper QL ring gained
    // nothing from spreading.)
    static constexpr int KS = BK / 32;
    static constexpr int FIT = (LOADS + TM * TN - 1) / (TM * TN);
    static constexpr int ISSUE_STEPS = (STAGES > 2 || DX > 0) ? KS : (FIT < KS ? FIT : KS);
    static_assert(QL_WAIT < 64, "vmcnt range");
    static_assert(STAGES >= 2, "one tile in flight while one is consumed");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS");
};

// Workgroup w covers tile tile_of(w) and, with split-K, the k-tiles
// [split * kts, split * kts + kts) of its piece.
template <class T, bool GATHER, int MODE, bool NTD>
__global__ __launch_bounds__(T::THREADS) void k_gemm_ring(const uint8_t* __restrict__ D,
                                                          uint64_t pitch,
                                                          const int8_t* __restrict__ QL,
                                                          uint32_t Cp, uint32_t n_tiles,
                                                          uint32_t m_tiles, uint32_t kts, Epi e) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const uint32_t R = e.R, C = e.C, M = e.M;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / T::WN;
    const int wn = wave % T::WN;

    const TileId tl = tile_of(xcd_remap(blockIdx.x, gridDim.x), n_tiles, m_tiles,
                              GATHER ? m_tiles : 8u);
    const uint32_t m0 = tl.m * T::BM;
    const uint32_t n0 = tl.n * T::BN;
    const uint32_t ktiles_all = (C + T::BK - 1) / T::BK;
    const uint32_t kt0 = tl.split * kts;
    const uint32_t ktiles = kt0 < ktiles_all ? min(kts, ktiles_all - kt0) : 0u;

    // Per-lane source of each of this wave's LOADS block loads: lane l of a
    // load fills slot l % SEGS of row l / SEGS of a 1 KiB block.  Loads
    // i < A_LOADS carry D rows, the rest QL rows.
    const int lrow = lane / T::SEGS;
    const uint8_t* src[T::LOADS];
    uint32_t seg_off[T::LOADS];
    // Load i of a stage's list: a D load (is_a) and its block index within
    // the D or QL part of the tile.
    auto is_a = [](int i) { return T::DX > 0 ? i >= T::B_LOADS : i < T::A_LOADS; };
    auto blk = [](int i) {
        return T::DX > 0 ? (i >= T::B_LOADS ? i - T::B_LOADS : i)
                         : (i < T::A_LOADS ? i : i - T::A_LOADS);
    };
#pragma unroll
    for (int i = 0; i < T::LOADS; ++i) {
        const bool a = is_a(i);
        const int kb = wave + T::NW * blk(i);
        const int r = kb * T::RPB + lrow;
        const int seg = swz<T::BK>(r, lane % T::SEGS);
        seg_off[i] = 16u * seg;
        if (a) {
            uint32_t mi = m0 + r;
            mi = mi < M ? mi : M - 1;
            uint32_t dr = GATHER ? e.rows[mi] : mi;
            dr = dr < R ? dr : R - 1;
            src[i] = D + (uint64_t)dr * pitch;
        } else {
            src[i] = reinterpret_cast<const uint8_t*>(QL) + ql_row(n0 + r, Cp) + seg_off[i];
        }
    }

    // Load i of k-tile t into its ring slot.  Every load is issued, so each
    // wave has the same count in flight per tile:
    // * a D segment past column C reads the row's last 16 bytes instead (C
    //   is a multiple of 16); those bytes meet zero-padded query bytes;
    // * t past the piece's last tile is clamped to it: such a load refills a
    //   slot no later iteration reads.
    const uint32_t t_last = ktiles ? ktiles - 1 : 0;
    uint8_t* const ringA = smem;                          // SA D tiles
    uint8_t* const ringB = smem + T::SA * T::A_BYTES;     // SB QL tiles
    // Load i of the list issued at stage u: D tile u + SA - 1 or QL tile
    // u + SB - 1 (DX == 0: the same tile u + STAGES - 1).
    auto issue_tile = [&](uint32_t t, int i) {
        const bool a = is_a(i);
        const uint32_t tt = min(t, t_last);
        const uint32_t k0 = (kt0 + tt) * T::BK;
        uint8_t* dst = (a ? ringA + (t % T::SA) * T::A_BYTES : ringB + (t % T::SB) * T::B_BYTES) +
                       (wave + T::NW * blk(i)) * 1024;
        const uint8_t* p = a ? src[i] + min(k0 + seg_off[i], C - 16u)
                             : src[i] + ql_col(k0);   // BK divides 128
        if (NTD && a)   // D read once: non-temporal
            __builtin_amdgcn_global_load_lds((glb_void_t*)p, (lds_void_t*)dst, 16, 0, kCpolNT);
        else
            __builtin_amdgcn_global_load_lds((glb_void_t*)p, (lds_void_t*)dst, 16, 0, 0);
    };
    auto issue_one = [&](uint32_t u, int i) {
        issue_tile(u + (is_a(i) ? T::SA : T::SB) - 1, i);
    };

    i32x16 acc[T::TM][T::TN];
#pragma unroll
    for (int a = 0; a < T::TM; ++a)
#pragma unroll
        for (int b = 0; b < T::TN; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[a][b][v] = 0;

    const int frow = lane & 31;
    const int fseg = lane >> 5;
    const u32x4 centre = u32x4{kCentreWord, kCentreWord, kCentreWord, kCentreWord};
    constexpr int KS = T::KS;

    // Fragments of one k-step of tile u (buffer buf).
    u32x4 fa[2][T::TM];
    i32x4 fb[2][T::TN];
    auto read_frags = [&](uint32_t u, int ks, int buf) {
        const uint8_t* sa = ringA + (u % T::SA) * T::A_BYTES;
        const uint8_t* sb = ringB + (u % T::SB) * T::B_BYTES;
        const int seg = 2 * ks + fseg;
#pragma unroll
        for (int a = 0; a < T::TM; ++a) {
            const int r = wm * T::TM * 32 + a * 32 + frow;
            fa[buf][a] = *reinterpret_cast<const u32x4*>(sa + r * T::BK + 16 * swz<T::BK>(r, seg));
        }
#pragma unroll
        for (int b = 0; b < T::TN; ++b) {
            const int r = wn * T::TN * 32 + b * 32 + frow;
            fb[buf][b] = *reinterpret_cast<const i32x4*>(sb + r * T::BK + 16 * swz<T::BK>(r, seg));
        }
    };
    // One k-step of MFMAs (centred A fragments ac, B buffer buf) with loads
    // lo .. hi-1 of stage u's list placed between them, one after each MFMA
    // (VMEM and MFMA scheduling groups); narrow tiles, with more loads than
    // MFMAs, issue the rest after the last MFMA.
    auto mfma_step = [&](const i32x4 (&ac)[T::TM], int buf, uint32_t u, int lo, int hi) {
        constexpr int kMfma = T::TM * T::TN;
#pragma unroll
        for (int a = 0; a < T::TM; ++a)
#pragma unroll
            for (int b = 0; b < T::TN; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ac[a], fb[buf][b], acc[a][b], 0, 0, 0);
#pragma unroll
        for (int i = lo; i < hi; ++i) issue_one(u, i);
        const int paired = hi - lo < kMfma ? hi - lo : kMfma;
#pragma unroll
        for (int j = 0; j < paired; ++j) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x010, 1, 0);
        }
#pragma unroll
        for (int j = paired; j < kMfma; ++j) __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
#pragma unroll
        for (int j = paired; j < hi - lo; ++j) __builtin_amdgcn_sched_group_barrier(0x010, 1, 0);
        __builtin_amdgcn_sched_barrier(0);
    };
    // First load of tile t_next issued in k-step j.
    auto first_load = [](int j) {
        return j < T::ISSUE_STEPS ? j * T::LOADS / T::ISSUE_STEPS : T::LOADS;
    };

    // The lists of the stages before the first, in the same order: stage v
    // (v = -(max(SA, SB)-1) .. -1) issues the tiles of its list that exist.
    if (ktiles > 0) {
#pragma unroll
        for (int v = -(T::SMAX - 1); v < 0; ++v)
#pragma unroll
            for (int i = 0; i < T::LOADS; ++i) {
                const int t = v + (is_a(i) ? T::SA : T::SB) - 1;
                if (t >= 0) issue_tile((uint32_t)t, i);
            }
    }

    for (uint32_t u = 0; u < ktiles; ++u) {
        // The loads issued after tile u's (see QL_WAIT) may still be in
        // flight; loads complete in order, so tile u has landed once at most
        // that many of this wave's loads are outstanding.  The barrier then
        // makes every wave's part visible and frees the slots of tile u-1
        // (every wave's reads of it have returned: the last MFMAs of tile
        // u-1 waited for them), which are refilled with D tile u+SA-1 and
        // QL tile u+SB-1 while tile u is consumed.
        wait_vmcnt<T::QL_WAIT>();
        ring_barrier();

        // Per k-step: centre the A fragments, read the fragments of the next
        // step, then the MFMAs with this step's share of the next tile's
        // loads between them (ISSUE_STEPS).  A wave issuing a tile's loads
        // back to back waits on the address unit with no MFMA to run
        // (measured: about 40% of the loop); between MFMAs the waits overlap
        // them.  The scheduling barriers keep this order.
        read_frags(u, 0, 0);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            i32x4 a_c[T::TM];
#pragma unroll
            for (int a = 0; a < T::TM; ++a) a_c[a] = __builtin_bit_cast(i32x4, fa[ks & 1][a] ^ centre);
            __builtin_amdgcn_sched_barrier(0);
            if (ks + 1 < KS) read_frags(u, ks + 1, (ks + 1) & 1);
            __builtin_amdgcn_sched_barrier(0);
            mfma_step(a_c, ks & 1, u, first_load(ks), first_load(ks + 1));
        }
    }
    // Loads past the last tile may still be landing in LDS.
    wait_vmcnt<0>();

    if constexpr (T::NARROW)
        epi_wave_narrow<MODE, GATHER, T::TM, T::TN>(e, tl.split, acc, m0 + wm * T::TM * 32,
                                                     n0 + wn * T::TN * 32, lane);
    else
        epi_wave<MODE, GATHER, T::TM, T::TN>(e, tl.split, acc, m0 + wm * T::TM * 32,
                                              n0 + wn * T::TN * 32, lane);
}

// ---------------------------------------------------------------- GEMM, split load roles
// Vector-memory loads of one wave complete in order, so a wave that feeds
// both the D stream (HBM, long latency) and the query stream (L2, short
// latency) can only run as far ahead as the shorter ring allows.  Here waves
// 0-1 load only D tiles into a deep ring of SA stages and waves 2-3 load only
// query tiles into a ring of SB stages; each wave waits on its own counter,
// then all four meet at the barrier and compute.  LWE form, no split.
template <int WM_, int WN_, int TM_, int TN_, int SA_, int SB_>
struct Roles {
    static constexpr int WM = WM_, WN = WN_, TM = TM_, TN = TN_, SA = SA_, SB = SB_;
    static constexpr int BK = 64;
    static constexpr int BM = WM * TM * 32;
    static constexpr int BN = WN * TN * 32;
    static constexpr int A_BYTES = BM * BK;
    static constexpr int B_BYTES = BN * BK;
    static constexpr int A_LOADS = BM / 16 / 2;          // per loader wave per tile
    static constexpr int B_LOADS = BN / 16 / 2;
    static constexpr int LDS_BYTES = SA * A_BYTES + SB * B_BYTES;
    static_assert(WM * WN == 4, "four waves");
    static_assert(TN % 4 == 0, "a wave covers whole groups of four limbs");
    static_assert(SA >= 2 && SB >= 2, "at least double buffering");
    static_assert((SA - 2) * A_LOADS < 64 && (SB - 2) * B_LOADS < 64, "vmcnt range");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS");
};

template <class T, bool GATHER>
__global__ __launch_bounds__(256) void k_gemm_roles(const uint8_t* __restrict__ D, uint64_t pitch,
                                                    const int8_t* __restrict__ QL, uint32_t Cp,
                                                    uint32_t n_tiles, uint32_t m_tiles, Epi e) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const uint32_t R = e.R, C = e.C, M = e.M;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / T::WN;
    const int wn = wave % T::WN;
    const bool loads_d = wave < 2;
    const int lw = wave & 1;                               // index among the loader pair

    const TileId tl = tile_of(xcd_remap(blockIdx.x, gridDim.x), n_tiles, m_tiles);
    const uint32_t m0 = tl.m * T::BM;
    const uint32_t n0 = tl.n * T::BN;

    constexpr int NL = T::A_LOADS > T::B_LOADS ? T::A_LOADS : T::B_LOADS;
    const uint8_t* src[NL];
    uint32_t seg_off[NL];
    const int lrow = lane >> 2;
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int kb = lw + 2 * i;                         // 1 KiB block within the tile
        const int r = kb * 16 + lrow;
        const int seg = swz<64>(r, lane & 3);
        seg_off[i] = 16u * seg;
        if (loads_d) {
            uint32_t mi = m0 + (uint32_t)min(r, T::BM - 1);
            mi = mi < M ? mi : M - 1;
            uint32_t dr = GATHER ? e.rows[mi] : mi;
            dr = dr < R ? dr : R - 1;
            src[i] = D + (uint64_t)dr * pitch + seg_off[i];
        } else {
            src[i] = reinterpret_cast<const uint8_t*>(QL) +
                     ql_row(n0 + (uint32_t)min(r, T::BN - 1), Cp) + seg_off[i];
        }
    }
    const uint32_t ktiles = (C + T::BK - 1) / T::BK;
    uint8_t* ringA = smem;
    uint8_t* ringB = smem + T::SA * T::A_BYTES;

    auto issue = [&](uint32_t t) {
        const uint32_t k0 = t * T::BK;
        if (loads_d) {
            uint8_t* stage = ringA + (t % T::SA) * T::A_BYTES;
#pragma unroll
            for (int i = 0; i < T::A_LOADS; ++i) {
                uint8_t* dst = stage + (lw + 2 * i) * 1024;
                if (k0 + seg_off[i] + 16 <= C)
                    __builtin_amdgcn_global_load_lds((glb_void_t*)(src[i] + k0), (lds_void_t*)dst,
                                                     16, 0, 0);
            }
        } else {
            uint8_t* stage = ringB + (t % T::SB) * T::B_BYTES;
            const uint32_t kq = ql_col(k0);
#pragma unroll
            for (int i = 0; i < T::B_LOADS; ++i) {
                uint8_t* dst = stage + (lw + 2 * i) * 1024;
                __builtin_amdgcn_global_load_lds((glb_void_t*)(src[i] + kq), (lds_void_t*)dst,
                                                 16, 0, 0);
            }
        }
    };

    i32x16 acc[T::TM][T::TN];
#pragma unroll
    for (int a = 0; a < T::TM; ++a)
#pragma unroll
        for (int b = 0; b < T::TN; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[a][b][v] = 0;

    const int frow = lane & 31;
    const int fseg = lane >> 5;
    const u32x4 centre = u32x4{kCentreWord, kCentreWord, kCentreWord, kCentreWord};

    const int depth = loads_d ? T::SA : T::SB;
    for (int p = 0; p < depth - 1; ++p)
        if ((uint32_t)p < ktiles) issue(p);

    for (uint32_t t = 0; t < ktiles; ++t) {
        // Each loader wave waits for its own part of tile t (counting as in
        // k_gemm_ring; only D loads of the last tile can be skipped).
        if (loads_d) {
            if (t + T::SA - 1 < ktiles) wait_vmcnt<(T::SA - 2) * T::A_LOADS>();
            else wait_vmcnt<0>();
        } else {
            if (t + T::SB - 1 < ktiles) wait_vmcnt<(T::SB - 2) * T::B_LOADS>();
            else wait_vmcnt<0>();
        }
        ring_barrier();
        if (t + depth - 1 < ktiles) issue(t + depth - 1);

        const uint8_t* sa = ringA + (t % T::SA) * T::A_BYTES;
        const uint8_t* sb = ringB + (t % T::SB) * T::B_BYTES;
#pragma unroll
        for (int ks = 0; ks < T::BK / 32; ++ks) {
            const int seg = 2 * ks + fseg;
            i32x4 fa[T::TM], fb[T::TN];
#pragma unroll
            for (int a = 0; a < T::TM; ++a) {
                const int r = wm * T::TM * 32 + a * 32 + frow;
                u32x4 v = *reinterpret_cast<const u32x4*>(sa + r * T::BK + 16 * swz<64>(r, seg));
                v ^= centre;
                fa[a] = __builtin_bit_cast(i32x4, v);
            }
#pragma unroll
            for (int b = 0; b < T::TN; ++b) {
                const int r = wn * T::TN * 32 + b * 32 + frow;
                fb[b] = *reinterpret_cast<const i32x4*>(sb + r * T::BK + 16 * swz<64>(r, seg));
            }
#pragma unroll
            for (int a = 0; a < T::TM; ++a)
#pragma unroll
                for (int b = 0; b < T::TN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb[b], acc[a][b], 0, 0, 0);
        }
    }
    epi_wave<kFinal32, GATHER, T::TM, T::TN>(e, 0, acc, m0 + wm * T::TM * 32,
                                              n0 + wn * T::TN * 32, lane);
}

// ---------------------------------------------------------------- dispatch
struct Gemm {
    const pir_db_t* db;
    const int8_t* QL;
    uint32_t Cp, N;
    Epi e;
    uint32_t splits, kts;   // split-K pieces and k-tiles per piece
    bool exact;             // field form
};

uint32_t g_cus = 256;       // compute units of the device (set at init)
uint64_t g_max_grid_y = 65535;   // largest grid y extent of the device (set at init)

uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// With one column tile (a batch no wider than the tile), each byte of D is
// read by one workgroup only, so D's loads are marked non-temporal and do
// not evict the limb planes every workgroup re-reads.
template <class T, bool GATHER, int MODE>
pir_status launch_ring_mode(const Gemm& g, uint32_t n_tiles, uint32_t m_tiles, hipStream_t s) {
    const uint64_t blocks = (uint64_t)n_tiles * m_tiles * g.splits;
    if (blocks > 0x7FFFFFFFull) return PIR_ERR_SHAPE;
    bool nt = false;
    if constexpr (!GATHER) {
        if (n_tiles == 1) {
            nt = true;
            k_gemm_ring<T, false, MODE, true><<<(uint32_t)blocks, T::THREADS, T::LDS_BYTES, s>>>(
                g.db->D, g.db->pitch, g.QL, g.Cp, n_tiles, m_tiles, g.kts, g.e);
        }
    }
    if (!nt)
        k_gemm_ring<T, GATHER, MODE, false><<<(uint32_t)blocks, T::THREADS, T::LDS_BYTES, s>>>(
            g.db->D, g.db->pitch, g.QL, g.Cp, n_tiles, m_tiles, g.kts, g.e);
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

template <class T>
pir_status launch_ring(const Gemm& g, hipStream_t s) {
    const uint32_t n_tiles = ceil_div(g.N, T::BN);
    const uint32_t m_tiles = ceil_div(g.e.M, T::BM);
    const bool gather = g.e.rows != nullptr;
    if (g.exact) {
        if (gather) return PIR_ERR_UNSUPPORTED;
        if (g.splits > 1) return launch_ring_mode<T, false, kPart64>(g, n_tiles, m_tiles, s);
        return launch_ring_mode<T, false, kFinalModP>(g, n_tiles, m_tiles, s);
    }
    if (g.splits > 1) {
        if (gather) return launch_ring_mode<T, true, kPart32>(g, n_tiles, m_tiles, s);
        return launch_ring_mode<T, false, kPart32>(g, n_tiles, m_tiles, s);
    }
    if (gather) return launch_ring_mode<T, true, kFinal32>(g, n_tiles, m_tiles, s);
    return launch_ring_mode<T, false, kFinal32>(g, n_tiles, m_tiles, s);
}

template <class T>
pir_status set_ring_lds() {
    const void* fns[] = {
        (const void*)k_gemm_ring<T, false, kFinal32, false>,
        (const void*)k_gemm_ring<T, true, kFinal32, false>,
        (const void*)k_gemm_ring<T, false, kPart32, false>,
        (const void*)k_gemm_ring<T, true, kPart32, false>,
        (const void*)k_gemm_ring<T, false, kPart64, false>,
        (const void*)k_gemm_ring<T, false, kFinalModP, false>,
        (const void*)k_gemm_ring<T, false, kFinal32, true>,
        (const void*)k_gemm_ring<T, false, kPart32, true>,
        (const void*)k_gemm_ring<T, false, kPart64, true>,
        (const void*)k_gemm_ring<T, false, kFinalModP, true>,
    };
    for (const void* f : fns)
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, T::LDS_BYTES) !=
            hipSuccess)
            return PIR_ERR_DEVICE;
    return PIR_OK;
}

template <class T>
pir_status launch_roles(const Gemm& g, hipStream_t s) {
    if (g.exact || g.splits != 1) return PIR_ERR_UNSUPPORTED;
    const uint32_t n_tiles = ceil_div(g.N, T::BN);
    const uint32_t m_tiles = ceil_div(g.e.M, T::BM);
    const uint64_t blocks = (uint64_t)n_tiles * m_tiles;
    if (blocks > 0x7FFFFFFFull) return PIR_ERR_SHAPE;
    if (g.e.rows)
        k_gemm_roles<T, true><<<(uint32_t)blocks, 256, T::LDS_BYTES, s>>>(
            g.db->D, g.db->pitch, g.QL, g.Cp, n_tiles, m_tiles, g.e);
    else
        k_gemm_roles<T, false><<<(uint32_t)blocks, 256, T::LDS_BYTES, s>>>(
            g.db->D, g.db->pitch, g.QL, g.Cp, n_tiles, m_tiles, g.e);
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

template <class T>
pir_status set_roles_lds() {
    if (hipFuncSetAttribute((const void*)k_gemm_roles<T, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, T::LDS_BYTES) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_gemm_roles<T, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, T::LDS_BYTES) != hipSuccess)
        return PIR_ERR_DEVICE;
    return PIR_OK;
}

template <class T>
pir_status launch_reg(const Gemm& g, hipStream_t s) {
    if (g.exact || g.splits != 1) return PIR_ERR_UNSUPPORTED;
    const uint32_t n_tiles = ceil_div(g.N, T::BN);
    const uint32_t m_tiles = ceil_div(g.e.M, T::BM);
    const uint64_t blocks = (uint64_t)n_tiles * m_tiles;
    if (blocks > 0x7FFFFFFFull) return PIR_ERR_SHAPE;
    const pir_db_t* db = g.db;
#define PIR_GEMM(VEC, GATHER)                                                              \
    k_gemm<T, VEC, GATHER><<<(uint32_t)blocks, 256, 0, s>>>(db->D, db->pitch, g.QL, g.Cp, \
                                                             n_tiles, g.e)
    const bool gather = g.e.rows != nullptr;
    if (db->aligned) {
        if (gather) PIR_GEMM(true, true); else PIR_GEMM(true, false);
    } else {
        if (gather) PIR_GEMM(false, true); else PIR_GEMM(false, false);
    }
#undef PIR_GEMM
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

// Kernel variants of the batched product.  Ring and roles variants need a
// 16-byte aligned database with C a multiple of 16; 256-wide tiles need N a
// multiple of 256 (batches above 32 queries, padded to 64).  Only ring
// variants split K (and so serve the field form).
using Ring128x128S8 = Ring<4, 1, 1, 4, 8>;              // 128 KiB LDS
using Ring128x128K128S4 = Ring<4, 1, 1, 4, 4, 128>;     // 128 KiB, 128-byte stages
using Ring128x256S6 = Ring<2, 2, 2, 4, 6>;              // 144 KiB
using Ring8w128x256K128S3 = Ring<4, 2, 1, 4, 3, 128>;   // 8 waves, 144 KiB
using Ring8w256x256S4 = Ring<4, 2, 2, 4, 4>;            // 8 waves, 128 KiB
using Ring8w256x256K128S2 = Ring<4, 2, 2, 4, 2, 128>;   // 8 waves, 128 KiB
// The same with a third D slot (D two tiles ahead, QL one): 160 KiB.
using Ring8w256x256K128D3 = Ring<4, 2, 2, 4, 2, 128, false, 1>;
// 128 x 256 with four D slots and three QL slots: 160 KiB.
using Ring8w128x256K128D4 = Ring<4, 2, 1, 4, 3, 128, false, 1>;
// 128 x 256 with five D slots (D four tiles ahead) and two QL slots: 144 KiB.
using Ring8w128x256K128D5 = Ring<4, 2, 1, 4, 2, 128, false, 3>;
// 256 x 256 with a third QL slot (limb planes two tiles ahead): 160 KiB.
using Ring8w256x256K128Q3 = Ring<4, 2, 2, 4, 2, 128, false, 0, 1>;
// Narrow tiles with deeper D rings: 256 x 32 with 4 D / 3 QL slots (140 KiB),
// 128 x 32 with 8 D / 6 QL slots (152 KiB).
using Narrow256x32K128D4 = Ring<4, 1, 2, 1, 3, 128, true, 1>;
using Narrow128x32K128D8 = Ring<4, 1, 1, 1, 6, 128, true, 2>;
using Ring256x256K128S2 = Ring<2, 2, 4, 4, 2, 128>;     // 4 waves of 128 x 128, 128 KiB
// The same with the D or the limb-plane ring one tile deeper (160 KiB): a
// 128 x 128 wave tile reads 0.5 KiB of LDS fragments per MFMA against 0.75
// for the 8-wave tile's 64 x 128.
using Ring256x256K128D3 = Ring<2, 2, 4, 4, 2, 128, false, 1>;
using Ring256x256K128Q3 = Ring<2, 2, 4, 4, 2, 128, false, 0, 1>;
// Two workgroups per CU (64 KiB each): the waves sharing a SIMD belong to
// different workgroups, so one's barrier does not idle the other.
using Ring128x128K128S2 = Ring<4, 1, 1, 4, 2, 128>;
// Narrow layout (8 queries per 32-column tile), one column tile per batch.
using Narrow256x32K128S4 = Ring<4, 1, 2, 1, 4, 128, true>;    // <= 8 queries, 144 KiB
using Narrow256x64K128S4 = Ring<8, 1, 1, 2, 4, 128, true>;    // <= 16 queries, 160 KiB
using Narrow128x32K128S6 = Ring<4, 1, 1, 1, 6, 128, true>;    // <= 8 queries, 120 KiB
using Roles256x256A5B4 = Roles<2, 2, 4, 4, 5, 4>;       // 80 + 64 KiB
using Roles128x256A10B4 = Roles<2, 2, 2, 4, 10, 4>;     // 80 + 64 KiB
using Reg128x256 = Tile<2, 2, 2, 4, 128>;
using Reg128x128 = Tile<4, 1, 1, 4, 128>;

enum Kind : uint8_t { kAuto, kRing, kRoles, kReg, kFew };

struct VariantInfo {
    const char* name;
    Kind kind;
    uint32_t bm, bn, bk;
    pir_status (*launch)(const Gemm&, hipStream_t);
    uint32_t per_cu;        // workgroups resident per CU (LDS-limited ring variants)
    bool narrow;            // narrow QL layout: all queries in one column tile
};

constexpr VariantInfo kVariants[] = {
    {"auto", kAuto, 0, 0, 0, nullptr},
    {"ring_128x128_s8", kRing, 128, 128, 64, launch_ring<Ring128x128S8>},
    {"ring_128x128_k128_s4", kRing, 128, 128, 128, launch_ring<Ring128x128K128S4>},
    {"ring_128x256_s6", kRing, 128, 256, 64, launch_ring<Ring128x256S6>},
    {"ring8w_128x256_k128_s3", kRing, 128, 256, 128, launch_ring<Ring8w128x256K128S3>},
    {"ring8w_256x256_s4", kRing, 256, 256, 64, launch_ring<Ring8w256x256S4>},
    {"ring8w_256x256_k128_s2", kRing, 256, 256, 128, launch_ring<Ring8w256x256K128S2>},
    {"ring_256x256_k128_s2", kRing, 256, 256, 128, launch_ring<Ring256x256K128S2>},
    {"roles_256x256_a5b4", kRoles, 256, 256, 64, launch_roles<Roles256x256A5B4>},
    {"roles_128x256_a10b4", kRoles, 128, 256, 64, launch_roles<Roles128x256A10B4>},
    {"reg_128x256", kReg, 128, 256, 128, launch_reg<Reg128x256>},
    {"reg_128x128", kReg, 128, 128, 128, launch_reg<Reg128x128>},
    {"few", kFew, 0, 0, 0, nullptr},   // dot4 stream, batches of at most kFewMax
    {"ring_128x128_k128_s2", kRing, 128, 128, 128, launch_ring<Ring128x128K128S2>, 2},
    {"narrow_256x32_k128_s4", kRing, 256, 32, 128, launch_ring<Narrow256x32K128S4>, 1, true},
    {"narrow_256x64_k128_s4", kRing, 256, 64, 128, launch_ring<Narrow256x64K128S4>, 1, true},
    {"narrow_128x32_k128_s6", kRing, 128, 32, 128, launch_ring<Narrow128x32K128S6>, 1, true},
    {"ring8w_256x256_k128_d3q2", kRing, 256, 256, 128, launch_ring<Ring8w256x256K128D3>},
    {"ring8w_128x256_k128_d4q3", kRing, 128, 256, 128, launch_ring<Ring8w128x256K128D4>},
    {"ring8w_128x256_k128_d5q2", kRing, 128, 256, 128, launch_ring<Ring8w128x256K128D5>},
    {"ring8w_256x256_k128_d2q3", kRing, 256, 256, 128, launch_ring<Ring8w256x256K128Q3>},
    {"narrow_256x32_k128_d4q3", kRing, 256, 32, 128, launch_ring<Narrow256x32K128D4>, 1, true},
    {"narrow_128x32_k128_d8q6", kRing, 128, 32, 128, launch_ring<Narrow128x32K128D8>, 1, true},
    {"ring_256x256_k128_d3q2", kRing, 256, 256, 128, launch_ring<Ring256x256K128D3>},
    {"ring_256x256_k128_d2q3", kRing, 256, 256, 128, launch_ring<Ring256x256K128Q3>},
};
constexpr uint32_t kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);
constexpr uint32_t kVarRing128 = 2, kVarRing256 = 4, kVarReg256 = 10,
                   kVarReg128 = 11, kVarFew = 12, kVarRing4wD3 = 23;
constexpr bool same_name(const char* a, const char* b) {
    return *a == *b && (*a == '\0' || same_name(a + 1, b + 1));
}
// The built-in choices name table rows by index: keep them on their rows.
static_assert(same_name(kVariants[kVarRing128].name, "ring_128x128_k128_s4") &&
                  same_name(kVariants[kVarRing256].name, "ring8w_128x256_k128_s3") &&
                  same_name(kVariants[kVarReg256].name, "reg_128x256") &&
                  same_name(kVariants[kVarReg128].name, "reg_128x128") &&
                  same_name(kVariants[kVarFew].name, "few") &&
                  same_name(kVariants[kVarRing4wD3].name, "ring_256x256_k128_d3q2"),
              "default variant indices");

bool ring_ok(const pir_db_t* db) { return db->aligned && (db->cols % 16 == 0); }

uint32_t padded_batch(uint32_t B) { return B <= 32u ? 32u : (B + 63u) / 64u * 64u; }

// Queries a variant's QL layout holds for batch B: narrow variants hold one
// column tile (BN / 4 queries), the others B padded to 32 or to 64.
uint32_t layout_batch(const VariantInfo& vi, uint32_t B) {
    return vi.narrow ? vi.bn / 4u : padded_batch(B);
}

bool variant_valid(const pir_db_t* db, uint32_t B, uint32_t v) {
    if (v == 0) return true;
    if (v >= kNumVariants) return false;
    const VariantInfo& vi = kVariants[v];
    if (vi.kind == kFew) return B <= kFewMax;
    if (vi.kind != kReg && !ring_ok(db)) return false;
    if (vi.narrow) return 4u * B <= vi.bn;
    return (4u * padded_batch(B)) % vi.bn == 0;
}

// Matrix-core choice (any batch size, gathered rows allowed).  From 64
// queries up, the four-wave 256 x 256 tile with the deeper D ring
// (ring_256x256_k128_d3q2), which led the autotuner at 64-1024 queries on
// 32768^2, 131072^2, 65536 x 32768 and the 3072 x 2^18 field form.
uint32_t default_gemm(const pir_db_t* db, uint32_t B) {
    const uint32_t Bp = padded_batch(B);
    if (!ring_ok(db)) return Bp == 32u ? kVarReg128 : kVarReg256;
    if (Bp == 32u) return kVarRing128;
    return kVarRing4wD3;
}

// The dot4 stream beats the padded matrix-core tile up to two queries; at
// four it is bound by VALU issue (measured at 32768 x 32768: 173 vs 254 us
// for one query, 194 vs 236 us for two, 400 vs 224 us for four).
constexpr uint32_t kFewDefault = 2;

uint32_t default_variant(const pir_db_t* db, uint32_t B) {
    return B <= kFewDefault ? kVarFew : default_gemm(db, B);
}

// Gathered rows (the incremental hint): scattered row addresses add
// address-translation latency, which the three-stage 128 x 256 ring hides
// best.  Whole call, 1311 scattered rows of the 131072 x 131072 database,
// n = 1024, on two machines: 1001-1019 us, against 1007-1294 us for the
// two-stage 256 x 256 tile that is fastest over the whole database (that
// one took 1146 us for the same rows sorted, 980 us for consecutive rows).
uint32_t default_rows(const pir_db_t* db, uint32_t B) {
    return ring_ok(db) && padded_batch(B) >= 64u ? kVarRing256 : default_gemm(db, B);
}

struct SplitPlan {
    uint32_t splits, kts;
};

// Split-K plan for a ring variant.  LDS lets one or two ring workgroups
// (per_cu) reside on a CU, so a launch runs in ceil(tiles * S / slots)
// rounds of 1/S of the K range each, slots = CUs * per_cu; pick the S (up
// to kMaxSplits, at least two k-tiles per
// piece) that minimises that time, with a small charge per piece for the
// partials and the pipeline fill, considered only below two rounds of
// tiles.  The field form also caps each piece at kExactSpan columns.
SplitPlan plan_splits(uint32_t M, uint32_t N, uint32_t C, const VariantInfo& vi, bool exact) {
    const uint32_t ktiles = ceil_div(C, vi.bk);
    if (vi.kind != kRing || ktiles == 0) return {1u, ktiles};
    const uint64_t tiles = (uint64_t)ceil_div(M, vi.bm) * ceil_div(N, vi.bn);
    const uint32_t lo = exact ? ceil_div(ktiles, kExactSpan / vi.bk) : 1u;
    const uint64_t slots = (uint64_t)g_cus * std::max(1u, vi.per_cu);
    uint32_t best = lo;
    if (tiles < 2ull * slots) {
        const uint32_t hi = std::max(lo, std::min(kMaxSplits, ktiles / 2));
        double best_t = 1e30;
        for (uint32_t sp = lo; sp <= hi; ++sp) {
            const double t = (double)ceil_div(tiles * sp, slots) / sp + 0.005 * sp;
            if (t < best_t) {
                best_t = t;
                best = sp;
            }
        }
    }
    const uint32_t kts = ceil_div(ktiles, best);
    return {ceil_div(ktiles, kts), kts};
}

struct BatchLayout {
    uint32_t Bp, N, Cp;     // queries in the QL layout, its limb rows, padded columns
    size_t colsum_off, part_off, total;
};

// Largest (splits x output rows) of any split-K plan for the batches whose
// wide layout has N limb columns: every ring variant valid for them (narrow
// variants, one column tile, for N = 128: batches of at most 32), every
// output row count up to R (gathered calls have fewer rows, and so may split
// more), both forms.
uint64_t worst_split_rows(const pir_db_t* db, uint32_t N_wide) {
    const uint32_t R = (uint32_t)db->rows, C = (uint32_t)db->cols;
    const bool exact_ok = C <= kMaxExactCols;
    uint64_t worst = 0;   // splits x rows
    for (uint32_t v = 1; v < kNumVariants; ++v) {
        const VariantInfo& vi = kVariants[v];
        if (vi.kind != kRing) continue;
        if (vi.narrow ? N_wide != 128u : N_wide % vi.bn != 0) continue;
        const uint32_t N = vi.narrow ? vi.bn : N_wide;
        const uint32_t nt = N / vi.bn;
        const uint32_t mt_all = ceil_div(R, vi.bm);
        // Row counts where the plan may split for occupancy, then R itself.
        const uint64_t slots = (uint64_t)g_cus * std::max(1u, vi.per_cu);
        const uint32_t mt_hi = std::min<uint64_t>(mt_all, (2ull * slots + nt - 1) / nt);
        for (uint32_t mt = 1; mt <= mt_hi + 1 && mt <= mt_all; ++mt) {
            const uint32_t M = mt == mt_all ? R : mt * vi.bm;
            for (int x = 0; x <= (exact_ok ? 1 : 0); ++x) {
                const SplitPlan sp = plan_splits(M, N, C, vi, x == 1);
                if (sp.splits > 1) worst = std::max<uint64_t>(worst, (uint64_t)sp.splits * M);
            }
        }
        for (int x = 0; x <= (exact_ok ? 1 : 0); ++x) {
            const SplitPlan sp = plan_splits(R, N, C, vi, x == 1);
            if (sp.splits > 1) worst = std::max<uint64_t>(worst, (uint64_t)sp.splits * R);
        }
    }
    return worst;
}

// Split-K partial bytes the workspace reserves for batch B (8 bytes per
// partial).  The scan above costs tens of microseconds, so its result is
// kept in the handle per padded-batch bucket (racing writers store the same
// value).
size_t partial_bound(const pir_db_t* db, uint32_t B, uint32_t N) {
    if (!ring_ok(db)) return 0;
    std::atomic<uint64_t>& slot = db->split_rows[batch_bucket(N / 4)];
    uint64_t cached = slot.load(std::memory_order_relaxed);
    uint64_t worst;
    if (cached != 0 && (cached >> 40) == N) {
        worst = cached & ((1ull << 40) - 1);
    } else {
        worst = worst_split_rows(db, N);
        slot.store(((uint64_t)N << 40) | worst, std::memory_order_relaxed);
    }
    return worst ? round_up((size_t)worst * B * 8, kWsAlign) : 0;
}

// Workspace: limb planes, exact column sums, split-K partials.  The
// partial bound covers every variant (it depends on the wide layout only),
// and the wide layout's limb planes are the larger, so mfma_workspace_bytes
// uses the wide layout.
BatchLayout batch_layout(const pir_db_t* db, uint32_t B, const VariantInfo& vi) {
    BatchLayout L;
    L.Bp = layout_batch(vi, B);
    L.N = 4u * L.Bp;
    L.Cp = (uint32_t)round_up(db->cols, kKPad);
    L.colsum_off = round_up((size_t)L.N * L.Cp, kWsAlign);
    L.part_off = L.colsum_off + round_up((size_t)L.Bp * 8, kWsAlign);
    L.total = L.part_off + partial_bound(db, B, 4u * padded_batch(B));
    return L;
}

}  // namespace

pir_status mfma_init() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cus > 0)
        g_cus = (uint32_t)cus;
    int gy = 0;
    if (hipDeviceGetAttribute(&gy, hipDeviceAttributeMaxGridDimY, dev) == hipSuccess && gy > 0)
        g_max_grid_y = (uint64_t)gy;
    pir_status st;
    if ((st = set_ring_lds<Ring128x128S8>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring128x128K128S4>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring128x256S6>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring8w128x256K128S3>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring8w256x256S4>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring8w256x256K128S2>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring256x256K128S2>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring128x128K128S2>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Narrow256x32K128S4>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Narrow256x64K128S4>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Narrow128x32K128S6>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring8w256x256K128D3>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring8w128x256K128D4>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring8w128x256K128D5>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring8w256x256K128Q3>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Narrow256x32K128D4>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Narrow128x32K128D8>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring256x256K128D3>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring256x256K128Q3>()) != PIR_OK) return st;
    if ((st = set_roles_lds<Roles256x256A5B4>()) != PIR_OK) return st;
    return set_roles_lds<Roles128x256A10B4>();
}

uint32_t mfma_variant_count() { return kNumVariants; }

const char* mfma_variant_name(uint32_t v) { return v < kNumVariants ? kVariants[v].name : nullptr; }

bool mfma_variant_valid(const pir_db_t* db, uint32_t B, uint32_t v, bool gathered) {
    if (gathered && v != 0 && v < kNumVariants && kVariants[v].kind == kFew) return false;
    return variant_valid(db, B, v);
}

size_t mfma_workspace_bytes(const pir_db_t* db, uint32_t B) {
    if (B == 0) return 0;
    return std::max(batch_layout(db, B, kVariants[kVarRing128]).total, few_workspace_bytes(db, B));
}

// Every choice and every check of a batched call, before anything is
// enqueued: variant, layout, split plan, grid limits and the workspace bytes
// the call touches.
pir_status mfma_plan_batch(const pir_db_t* db, uint32_t B, const uint32_t* rows, uint32_t m,
                           uint32_t modulus, bool planes, BatchPlan* plan) {
    const uint32_t C = (uint32_t)db->cols;
    const bool exact = modulus != 0;
    if (exact && rows) return PIR_ERR_UNSUPPORTED;   // no gathered field form
    if (exact && C > kMaxExactCols) return PIR_ERR_SHAPE;
    if (exact && planes) return PIR_ERR_UNSUPPORTED;

    uint32_t v = (rows ? db->variant_rows : db->variant)[batch_bucket(B)];
    if (v == 0 || !variant_valid(db, B, v)) v = rows ? default_rows(db, B) : default_variant(db, B);
    if (rows && kVariants[v].kind == kFew) v = default_gemm(db, B);
    // Pre-ingested planes are in the wide layout: matrix-core variants that read it.
    if (planes && (kVariants[v].kind == kFew || kVariants[v].narrow)) v = default_gemm(db, B);
    if (exact && kVariants[v].kind != kRing && kVariants[v].kind != kFew)
        v = (B <= kFewDefault || (B <= kFewMax && !ring_ok(db))) ? kVarFew : default_gemm(db, B);
    if (exact && (kVariants[v].kind == kReg || kVariants[v].kind == kRoles ||
                  (kVariants[v].kind == kRing && !ring_ok(db))))
        return PIR_ERR_UNSUPPORTED;   // field form beyond kFewMax queries needs the ring kernels

    BatchPlan P{};
    P.variant = v;
    if (kVariants[v].kind == kFew) {
        P.few = true;
        P.need = few_workspace_bytes(db, B);
        *plan = P;
        return PIR_OK;
    }
    const VariantInfo& vi = kVariants[v];
    const BatchLayout L = batch_layout(db, B, vi);
    P.Bp = L.Bp;
    P.N = L.N;
    P.Cp = L.Cp;
    P.colsum_off = L.colsum_off;
    P.part_off = L.part_off;
    if ((uint64_t)L.Cp / kIngJ > g_max_grid_y) return PIR_ERR_SHAPE;   // ingest grid
    P.M = rows ? m : (uint32_t)db->rows;
    const SplitPlan sp = plan_splits(P.M, L.N, C, vi, exact);
    P.splits = sp.splits;
    P.kts = sp.kts;
    const uint64_t blocks = (uint64_t)ceil_div(L.N, vi.bn) * ceil_div(P.M, vi.bm) * sp.splits;
    if (blocks > 0x7FFFFFFFull) return PIR_ERR_SHAPE;
    P.need = L.part_off;
    if (sp.splits > 1) {
        const uint64_t n = (uint64_t)P.M * B;
        if ((n + 255) / 256 > 0x7FFFFFFFull) return PIR_ERR_SHAPE;   // k_finish grid
        P.need += (size_t)sp.splits * P.M * B * 8;
        if (P.need > L.total) return PIR_ERR_WORKSPACE;   // cannot happen: the layout bounds every plan
    }
    *plan = P;
    return PIR_OK;
}

// Zero the column sums, then write the limb planes and column sums of the
// queries into `base` (the layout of `P`).
static pir_status ingest(const pir_db_t* db, const BatchIO& io, uint32_t B, const BatchPlan& P,
                  bool narrow, uint8_t* base, hipStream_t s) {
    const uint32_t C = (uint32_t)db->cols;
    int8_t* QL = reinterpret_cast<int8_t*>(base);
    u64* colsum = reinterpret_cast<u64*>(base + P.colsum_off);
    k_zero_words<<<(2 * P.Bp + 255) / 256, 256, 0, s>>>(reinterpret_cast<uint32_t*>(colsum),
                                                         2 * P.Bp);
    PIR_LAUNCH_CHECK();
    dim3 ig((P.Bp + kIngB - 1) / kIngB, P.Cp / kIngJ);
    const bool qmajor = io.q_ldj == 1;
    const bool vec = ((uintptr_t)io.Q % 16 == 0) &&
                     (qmajor ? (io.q_ldb % 4 == 0 && C % 4 == 0) : (io.q_ldj % 4 == 0 && B % 4 == 0));
#define PIR_INGEST(QM, V)                                                                  \
    k_ingest<QM, V><<<ig, 256, 0, s>>>(io.Q, io.q_ldj, io.q_ldb, C, B, P.Bp, P.Cp, QL, colsum, \
                                       narrow)
    if (qmajor) {
        if (vec) PIR_INGEST(true, true); else PIR_INGEST(true, false);
    } else {
        if (vec) PIR_INGEST(false, true); else PIR_INGEST(false, false);
    }
#undef PIR_INGEST
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

// Enqueue a planned batched call; `ws` holds at least plan.need bytes.  With
// `planes` (the wide-layout limb planes and column sums of these queries,
// written by mfma_ingest_planes) the ingest is skipped.
pir_status mfma_run_batch(const pir_db_t* db, const BatchIO& io, uint32_t B,
                          const uint32_t* rows, uint32_t modulus, const BatchPlan& P, void* ws,
                          const void* planes, hipStream_t s) {
    if (P.few) return few_answer_batch(db, io, B, modulus, ws, P.need, s);
    const uint32_t C = (uint32_t)db->cols;
    const bool exact = modulus != 0;
    const VariantInfo& vi = kVariants[P.variant];
    uint8_t* base = static_cast<uint8_t*>(ws);
    const uint8_t* qbase = planes ? static_cast<const uint8_t*>(planes) : base;
    const int8_t* QL = reinterpret_cast<const int8_t*>(qbase);
    const u64* colsum = reinterpret_cast<const u64*>(qbase + P.colsum_off);
    if (!planes) {
        const pir_status st = ingest(db, io, B, P, vi.narrow, base, s);
        if (st != PIR_OK) return st;
    }
    if (P.M == 0) return PIR_OK;

    Gemm g;
    g.db = db;
    g.QL = QL;
    g.Cp = P.Cp;
    g.N = P.N;
    g.exact = exact;
    g.splits = P.splits;
    g.kts = P.kts;
    g.e = Epi{P.M,      B,        (uint32_t)db->rows, C, rows, colsum, db->rowsum, io.out,
              io.o_ldr, io.o_ldb, base + P.part_off, modulus};
    pir_status st = vi.launch(g, s);
    if (st != PIR_OK || P.splits <= 1) return st;
    const uint64_t n = (uint64_t)P.M * B;
    if (n == 0) return PIR_OK;
    const bool vec4 = !exact && B % 4 == 0 && io.o_ldb == 1 && io.o_ldr % 4 == 0 &&
                      (uintptr_t)io.out % 16 == 0;
    if (exact)
        k_finish<true><<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(g.e, P.splits);
    else if (vec4)
        k_finish4<<<(uint32_t)((n / 4 + 255) / 256), 256, 0, s>>>(g.e, P.splits);
    else
        k_finish<false><<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(g.e, P.splits);
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

pir_status mfma_answer_batch(const pir_db_t* db, const BatchIO& io, uint32_t B,
                             const uint32_t* rows, uint32_t m, uint32_t modulus, void* ws,
                             size_t ws_bytes, const void* planes, size_t planes_bytes,
                             hipStream_t s) {
    BatchPlan plan;
    const pir_status st = mfma_plan_batch(db, B, rows, m, modulus, planes != nullptr, &plan);
    if (st != PIR_OK) return st;
    // The reported size is the contract for every kernel path.
    if (!ws || ws_bytes < mfma_workspace_bytes(db, B) || ((uintptr_t)ws % kWsAlign))
        return PIR_ERR_WORKSPACE;
    if (planes && (planes_bytes < mfma_planes_bytes(db, B) || ((uintptr_t)planes % kWsAlign)))
        return PIR_ERR_WORKSPACE;
    return mfma_run_batch(db, io, B, rows, modulus, plan, ws, planes, s);
}

size_t mfma_planes_bytes(const pir_db_t* db, uint32_t n) {
    if (n == 0) return 0;
    return batch_layout(db, n, kVariants[kVarRing128]).part_off;
}

pir_status mfma_ingest_planes(const pir_db_t* db, const uint32_t* A, uint32_t n, void* planes,
                              size_t planes_bytes, hipStream_t s) {
    BatchLayout L = batch_layout(db, n, kVariants[kVarRing128]);
    if (!planes || planes_bytes < L.part_off || ((uintptr_t)planes % kWsAlign))
        return PIR_ERR_WORKSPACE;
    if ((uint64_t)L.Cp / kIngJ > g_max_grid_y) return PIR_ERR_SHAPE;
    BatchPlan P{};
    P.Bp = L.Bp;
    P.N = L.N;
    P.Cp = L.Cp;
    P.colsum_off = L.colsum_off;
    const BatchIO io{A, n, 1, nullptr, n, 1};
    return ingest(db, io, n, P, false, static_cast<uint8_t*>(planes), s);
}
