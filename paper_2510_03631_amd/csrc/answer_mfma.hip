// Batched Answer and offline hint on the int8 matrix cores.
//
//   Out[r][b] = sum_j D[r][j] * Q[j][b]  mod 2^32
//
// (the multi-request response of Section 5.2, Algorithm 4's batched product,
// here over Z/2^32; the hint H = D A is the same product with A in place of
// Q, Section 5.3's offline work).
//
// gfx950 has only signed int8 matrix instructions, so both operands are
// centred.  With q = sum_k 2^(8k) q_k (byte limbs), q_k = q'_k + 128 and
// D = D' + 128 (D' = D xor 0x80 read as int8, likewise q'_k):
//
//   D q = sum_k 2^(8k) (D' q'_k)  +  128 sum_k 2^(8k) colsum(q'_k)
//                                 +  0x80808080 rowsum(D)
//
// and sum_k 2^(8k) colsum(q'_k) = colsum(q) - C * 0x80808080.  So one int8
// GEMM with M = R, K = C and N = 4 * B (the four limb planes of every query
// side by side) gives the products P_k = D' q'_k; the epilogue adds
// P_0 + 2^8 P_1 + 2^16 P_2 + 2^24 P_3, the per-query column term and the
// per-row term kept in the database handle.  Every step is exact modulo
// 2^32: the int32 accumulators of the matrix instruction wrap modulo 2^32
// (two's complement), and only the residue is ever used.
//
// Kernels
//   k_zero_words  clear the column sums
//   k_ingest      Q (C x B words) -> QL (N x Cp centred int8, K-contiguous),
//                 colsum[b] += sum_j Q[j][b]
//   k_gemm        int8 MFMA 32x32x32 tiles, LDS double staging through
//                 registers, fused epilogue, optional row gather/scatter
//                 (the incremental hint touches only refreshed rows).
//
// QL row index of (query b, limb k): n = (b / 32) * 128 + k * 32 + (b % 32),
// so the four limbs of a query land in the same lane of four adjacent 32x32
// output tiles and the epilogue combines them in registers.
#include "qpir_internal.h"

namespace {

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

constexpr uint32_t kCentreWord = 0x80808080u;
constexpr int kKPad = 256;      // QL rows are padded with zeros to a multiple of this

__global__ void k_zero_words(uint32_t* __restrict__ p, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Block: 64 query coordinates j x 32 queries b.  Element (j, b) of the
// query matrix is Q[j * ldj + b * ldb].  The load is coalesced along b for
// the row-major layout (ldb == 1) and along j for the query-major one
// (QMAJOR, ldj == 1); both go through an LDS tile, then each thread writes
// 32 limb bytes of one query.
template <bool QMAJOR>
__global__ __launch_bounds__(256) void k_ingest(const uint32_t* __restrict__ Q, uint64_t ldj,
                                                uint64_t ldb, uint32_t C, uint32_t B, uint32_t Cp,
                                                int8_t* __restrict__ QL,
                                                uint32_t* __restrict__ colsum) {
    __shared__ uint32_t s[32][65];
    const int t = threadIdx.x;
    const uint32_t j0 = blockIdx.x * 64u;
    const uint32_t b0 = blockIdx.y * 32u;
    if (QMAJOR) {
        const int bb = t >> 3;
        const uint32_t b = b0 + bb;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const int jj = (t & 7) * 8 + p;
            const uint32_t j = j0 + jj;
            s[bb][jj] = (j < C && b < B) ? Q[(uint64_t)j * ldj + (uint64_t)b * ldb] : 0u;
        }
    } else {
        const int bb = t & 31;
        const uint32_t b = b0 + bb;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const int jj = (t >> 5) + 8 * p;
            const uint32_t j = j0 + jj;
            s[bb][jj] = (j < C && b < B) ? Q[(uint64_t)j * ldj + (uint64_t)b * ldb] : 0u;
        }
    }
    __syncthreads();
    const int limb = t >> 6;
    const int bb = (t >> 1) & 31;
    const int half = t & 1;
    const uint32_t b = b0 + bb;
    uint32_t w[8];
    uint32_t sum = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        uint32_t word = 0;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            const int jj = 32 * half + 4 * e + x;
            const uint32_t j = j0 + jj;
            const uint32_t v = s[bb][jj];
            sum += v;
            const uint32_t byte = (j < C && b < B) ? (((v >> (8 * limb)) & 0xFFu) ^ 0x80u) : 0u;
            word |= byte << (8 * x);
        }
        w[e] = word;
    }
    const uint32_t n = (b0 / 32u) * 128u + (uint32_t)limb * 32u + (uint32_t)bb;
    u32x4* dst = reinterpret_cast<u32x4*>(QL + (uint64_t)n * Cp + j0 + 32u * half);
    dst[0] = u32x4{w[0], w[1], w[2], w[3]};
    dst[1] = u32x4{w[4], w[5], w[6], w[7]};
    if (limb == 0) {
        sum += __shfl_xor(sum, 1);
        if (half == 0 && b < B) atomicAdd(&colsum[b], sum);
    }
}

// ---------------------------------------------------------------- GEMM
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
// (TM*32) x (TN*32) with 32x32x32 int8 MFMAs.
template <class T, bool VEC, bool GATHER>
__global__ __launch_bounds__(256) void k_gemm(const uint8_t* __restrict__ D, uint64_t pitch,
                                              uint32_t R, uint32_t C,
                                              const uint32_t* __restrict__ rows, uint32_t M,
                                              const int8_t* __restrict__ QL, uint32_t Cp,
                                              uint32_t B, uint32_t n_tiles,
                                              const uint32_t* __restrict__ colsum,
                                              const uint32_t* __restrict__ rowterm,
                                              uint32_t* __restrict__ out, uint64_t o_ldr,
                                              uint64_t o_ldb) {
    __shared__ __attribute__((aligned(16))) uint8_t sA[T::BM * T::LDK];
    __shared__ __attribute__((aligned(16))) uint8_t sB[T::BN * T::LDK];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / T::WN;
    const int wn = wave % T::WN;

    // Tiles are numbered n-fastest.  Consecutive workgroups are dealt to
    // the 8 XCDs in turn; remap so each XCD works on a contiguous range of
    // tiles (the row blocks of D it reads stay in its own L2).
    const uint32_t nblk = gridDim.x;
    uint32_t bid = blockIdx.x;
    {
        const uint32_t per = nblk / 8u;
        const uint32_t x = bid % 8u, l = bid / 8u;
        if (bid < per * 8u) bid = x * per + l;
    }
    const uint32_t tile_m = bid / n_tiles;
    const uint32_t tile_n = bid % n_tiles;
    const uint32_t m0 = tile_m * T::BM;
    const uint32_t n0 = tile_n * T::BN;

    // Global load assignment: thread -> (row, 16-byte segment).
    const int seg = tid % T::SEGS;
    const int rsub = tid / T::SEGS;
    constexpr int ROWS_PER_PASS = 256 / T::SEGS;

    const uint8_t* arow[T::A_LOADS];
#pragma unroll
    for (int p = 0; p < T::A_LOADS; ++p) {
        uint32_t i = m0 + rsub + p * ROWS_PER_PASS;
        i = i < M ? i : M - 1;
        const uint32_t r = GATHER ? rows[i] : i;
        arow[p] = D + (uint64_t)(r < R ? r : R - 1) * pitch;
    }
    const int8_t* brow[T::B_LOADS];
#pragma unroll
    for (int p = 0; p < T::B_LOADS; ++p)
        brow[p] = QL + (uint64_t)(n0 + rsub + p * ROWS_PER_PASS) * Cp;

    u32x4 ra[T::A_LOADS], rb[T::B_LOADS];
    auto gload = [&](uint32_t k0) {
        const uint32_t k = k0 + 16u * seg;
#pragma unroll
        for (int p = 0; p < T::A_LOADS; ++p) ra[p] = load_row16<VEC>(arow[p], k, C);
#pragma unroll
        for (int p = 0; p < T::B_LOADS; ++p)
            rb[p] = *reinterpret_cast<const u32x4*>(brow[p] + k);
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

    // Epilogue: combine limbs, add the centring terms, store.
    const uint32_t cterm_base = (uint32_t)C * kCentreWord;
#pragma unroll
    for (int g = 0; g < T::TN / 4; ++g) {
        const uint32_t bq = (n0 + wn * T::TN * 32) / 4u + 32u * g + (uint32_t)(lane & 31);
        const uint32_t colterm = 128u * (bq < B ? colsum[bq] - cterm_base : 0u);
#pragma unroll
        for (int a = 0; a < T::TM; ++a) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const uint32_t i = m0 + wm * T::TM * 32 + a * 32 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
                if (i < M && bq < B) {
                    const uint32_t r = GATHER ? rows[i] : i;
                    if (r < R) {
                        const uint32_t p0 = (uint32_t)acc[a][4 * g + 0][v];
                        const uint32_t p1 = (uint32_t)acc[a][4 * g + 1][v];
                        const uint32_t p2 = (uint32_t)acc[a][4 * g + 2][v];
                        const uint32_t p3 = (uint32_t)acc[a][4 * g + 3][v];
                        out[(uint64_t)r * o_ldr + (uint64_t)bq * o_ldb] =
                            p0 + (p1 << 8) + (p2 << 16) + (p3 << 24) + colterm + rowterm[r];
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------- GEMM, LDS ring
// The main kernel for aligned databases with C a multiple of 16.  Global
// tiles go straight to LDS with global_load_lds_dwordx4 (no register
// staging), into a ring of STAGES k-tiles of 64 bytes, so STAGES-1 tiles are
// in flight while one is consumed.  A 64-byte LDS row holds four 16-byte
// slots; slot = segment ^ ((row >> 1) & 3) keeps the fragment reads
// (one row per lane, same segment) free of bank conflicts.  Centring of D
// (xor 0x80) is applied to the A fragments in registers.
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

template <int WM_, int WN_, int TM_, int TN_, int STAGES_, int BK_ = 64>
struct Ring {
    static constexpr int WM = WM_, WN = WN_, TM = TM_, TN = TN_, STAGES = STAGES_;
    static constexpr int NW = WM * WN;                   // waves per workgroup
    static constexpr int THREADS = 64 * NW;
    static constexpr int BK = BK_;                       // k bytes per stage: 64 or 128
    static constexpr int SEGS = BK / 16;                 // 16-byte slots per LDS row
    static constexpr int RPB = 1024 / BK;                // rows per 1 KiB block
    static constexpr int BM = WM * TM * 32;
    static constexpr int BN = WN * TN * 32;
    static constexpr int A_BYTES = BM * BK;
    static constexpr int STAGE_BYTES = (BM + BN) * BK;
    static constexpr int A_BLOCKS = BM / RPB;            // 1 KiB blocks
    static constexpr int BLOCKS = (BM + BN) / RPB;
    static constexpr int LOADS = BLOCKS / NW;            // per wave per tile
    static constexpr int LDS_BYTES = STAGES * STAGE_BYTES;
    static_assert(BK == 64 || BK == 128, "64- or 128-byte stages");
    static_assert(NW == 4 || NW == 8, "four or eight waves");
    static_assert(TN % 4 == 0, "a wave covers whole groups of four limbs");
    static_assert(BLOCKS % NW == 0, "blocks split evenly over waves");
    static_assert((STAGES - 2) * LOADS < 64, "vmcnt range");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS");
};

// 16-byte slot of (row, segment) in an LDS row.  A fragment read has 32
// lanes on 32 consecutive rows at one segment; gfx950's LDS serves a
// 16-byte read 16 lanes at a time across 64 four-byte banks, so the 16 rows
// of a pass must land on 16 distinct 16-byte bank groups.  A 64-byte row
// spans 16 banks (row % 4 picks the quarter of the bank space), a 128-byte
// row 32 banks (row % 2); XORing the segment with the next row bits fills
// the remaining choices.  (Measured: the earlier swizzle, conflict-free for
// 8 lanes over 32 banks, spent half of the LDS cycles in bank conflicts.)
template <int BK>
__device__ inline int swz(int row, int seg) {
    return BK == 64 ? (seg ^ ((row >> 2) & 3)) : (seg ^ ((row >> 1) & 7));
}

__device__ inline int slot_of(int row, int seg) { return swz<64>(row, seg); }

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

template <class T, bool GATHER>
__global__ __launch_bounds__(T::THREADS) void k_gemm_ring(const uint8_t* __restrict__ D, uint64_t pitch,
                                                   uint32_t R, uint32_t C,
                                                   const uint32_t* __restrict__ rows, uint32_t M,
                                                   const int8_t* __restrict__ QL, uint32_t Cp,
                                                   uint32_t B, uint32_t n_tiles, uint32_t m_tiles,
                                                   const uint32_t* __restrict__ colsum,
                                                   const uint32_t* __restrict__ rowterm,
                                                   uint32_t* __restrict__ out, uint64_t o_ldr,
                                                   uint64_t o_ldb) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / T::WN;
    const int wn = wave % T::WN;

    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous range of tile indices, then order tiles in groups of 8 row
    // tiles so the ~32 workgroups an XCD runs at once share D and QL tiles
    // in its L2.
    uint32_t bid = blockIdx.x;
    {
        const uint32_t per = gridDim.x / 8u;
        if (bid < per * 8u) bid = (bid % 8u) * per + bid / 8u;
    }
    constexpr uint32_t kGroup = 8;
    const uint32_t group = bid / (kGroup * n_tiles);
    const uint32_t first_m = group * kGroup;
    const uint32_t gsize = min(m_tiles - first_m, kGroup);
    const uint32_t in_group = bid % (kGroup * n_tiles);
    const uint32_t tile_m = first_m + in_group % gsize;
    const uint32_t tile_n = in_group / gsize;
    const uint32_t m0 = tile_m * T::BM;
    const uint32_t n0 = tile_n * T::BN;

    // Per-lane source of each of this wave's LOADS block loads: lane l of a
    // load fills slot l % SEGS of row l / SEGS of a 1 KiB block.
    const int lrow = lane / T::SEGS;                      // row within a 1 KiB block
    const uint8_t* src[T::LOADS];
    uint32_t seg_off[T::LOADS];
    bool is_a[T::LOADS];
#pragma unroll
    for (int i = 0; i < T::LOADS; ++i) {
        const int kb = wave + T::NW * i;
        const bool a = kb < T::A_BLOCKS;
        const int r = (a ? kb : kb - T::A_BLOCKS) * T::RPB + lrow;
        const int seg = swz<T::BK>(r, lane % T::SEGS);
        is_a[i] = a;
        seg_off[i] = 16u * seg;
        if (a) {
            uint32_t mi = m0 + r;
            mi = mi < M ? mi : M - 1;
            uint32_t dr = GATHER ? rows[mi] : mi;
            dr = dr < R ? dr : R - 1;
            src[i] = D + (uint64_t)dr * pitch + seg_off[i];
        } else {
            src[i] = reinterpret_cast<const uint8_t*>(QL) + (uint64_t)(n0 + r) * Cp + seg_off[i];
        }
    }
    const uint32_t ktiles = (C + T::BK - 1) / T::BK;

    auto issue = [&](uint32_t t) {
        const uint32_t k0 = t * T::BK;
        uint8_t* stage = smem + (t % T::STAGES) * T::STAGE_BYTES;
#pragma unroll
        for (int i = 0; i < T::LOADS; ++i) {
            const int kb = wave + T::NW * i;
            uint8_t* dst = stage + kb * 1024;   // A blocks first, then B blocks
            // D segments past the last column are skipped (their LDS slots
            // keep old bytes, which meet zero query bytes); QL rows are
            // zero-padded to Cp and always loaded.
            if (!is_a[i] || k0 + seg_off[i] + 16 <= C)
                __builtin_amdgcn_global_load_lds((glb_void_t*)(src[i] + k0), (lds_void_t*)dst,
                                                 16, 0, 0);
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

#pragma unroll
    for (int p = 0; p < T::STAGES - 1; ++p)
        if ((uint32_t)p < ktiles) issue(p);

    for (uint32_t t = 0; t < ktiles; ++t) {
        // Tiles t+1 .. t+STAGES-2 were issued after tile t.  While none of
        // them is the last tile (whose D loads past column C may be skipped
        // by a whole wave, issuing fewer loads), tile t has landed once at
        // most (STAGES-2) * LOADS of this wave's loads are outstanding
        // (loads complete in order).  Otherwise wait for all.  The barrier
        // then makes every wave's part visible and frees the stage consumed
        // in the previous iteration.
        if (t + T::STAGES - 1 < ktiles) wait_vmcnt<(T::STAGES - 2) * T::LOADS>();
        else wait_vmcnt<0>();
        ring_barrier();
        if (t + T::STAGES - 1 < ktiles) issue(t + T::STAGES - 1);

        const uint8_t* sa = smem + (t % T::STAGES) * T::STAGE_BYTES;
        const uint8_t* sb = sa + T::A_BYTES;
        // Fragments of k-step ks+1 are read while the MFMAs of ks run.
        constexpr int KS = T::BK / 32;
        i32x4 fa[2][T::TM], fb[2][T::TN];
        auto read_frags = [&](int ks, int buf) {
            const int seg = 2 * ks + fseg;
#pragma unroll
            for (int a = 0; a < T::TM; ++a) {
                const int r = wm * T::TM * 32 + a * 32 + frow;
                u32x4 v = *reinterpret_cast<const u32x4*>(sa + r * T::BK + 16 * swz<T::BK>(r, seg));
                v ^= centre;
                fa[buf][a] = __builtin_bit_cast(i32x4, v);
            }
#pragma unroll
            for (int b = 0; b < T::TN; ++b) {
                const int r = wn * T::TN * 32 + b * 32 + frow;
                fb[buf][b] = *reinterpret_cast<const i32x4*>(sb + r * T::BK + 16 * swz<T::BK>(r, seg));
            }
        };
        read_frags(0, 0);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            if (ks + 1 < KS) read_frags(ks + 1, (ks + 1) & 1);
#pragma unroll
            for (int a = 0; a < T::TM; ++a)
#pragma unroll
                for (int b = 0; b < T::TN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[ks & 1][a], fb[ks & 1][b],
                                                                      acc[a][b], 0, 0, 0);
        }
    }

    const uint32_t cterm_base = C * kCentreWord;
#pragma unroll
    for (int g = 0; g < T::TN / 4; ++g) {
        const uint32_t bq = (n0 + wn * T::TN * 32) / 4u + 32u * g + (uint32_t)(lane & 31);
        const uint32_t colterm = 128u * (bq < B ? colsum[bq] - cterm_base : 0u);
#pragma unroll
        for (int a = 0; a < T::TM; ++a) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const uint32_t i = m0 + wm * T::TM * 32 + a * 32 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
                if (i < M && bq < B) {
                    const uint32_t r = GATHER ? rows[i] : i;
                    if (r < R) {
                        const uint32_t p0 = (uint32_t)acc[a][4 * g + 0][v];
                        const uint32_t p1 = (uint32_t)acc[a][4 * g + 1][v];
                        const uint32_t p2 = (uint32_t)acc[a][4 * g + 2][v];
                        const uint32_t p3 = (uint32_t)acc[a][4 * g + 3][v];
                        out[(uint64_t)r * o_ldr + (uint64_t)bq * o_ldb] =
                            p0 + (p1 << 8) + (p2 << 16) + (p3 << 24) + colterm + rowterm[r];
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------- GEMM, split load roles
// Vector-memory loads of one wave complete in order, so a wave that feeds
// both the D stream (HBM, long latency) and the query stream (L2, short
// latency) can only run as far ahead as the shorter ring allows.  Here waves
// 0-1 load only D tiles into a deep ring of SA stages and waves 2-3 load only
// query tiles into a ring of SB stages; each wave waits on its own counter,
// then all four meet at the barrier and compute.
template <int WM_, int WN_, int TM_, int TN_, int SA_, int SB_>
struct Split {
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
__global__ __launch_bounds__(256) void k_gemm_split(const uint8_t* __restrict__ D, uint64_t pitch,
                                                    uint32_t R, uint32_t C,
                                                    const uint32_t* __restrict__ rows, uint32_t M,
                                                    const int8_t* __restrict__ QL, uint32_t Cp,
                                                    uint32_t B, uint32_t n_tiles, uint32_t m_tiles,
                                                    const uint32_t* __restrict__ colsum,
                                                    const uint32_t* __restrict__ rowterm,
                                                    uint32_t* __restrict__ out, uint64_t o_ldr,
                                                    uint64_t o_ldb) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / T::WN;
    const int wn = wave % T::WN;
    const bool loads_d = wave < 2;
    const int lw = wave & 1;                               // index among the loader pair

    uint32_t bid = blockIdx.x;
    {
        const uint32_t per = gridDim.x / 8u;
        if (bid < per * 8u) bid = (bid % 8u) * per + bid / 8u;
    }
    constexpr uint32_t kGroup = 8;
    const uint32_t group = bid / (kGroup * n_tiles);
    const uint32_t first_m = group * kGroup;
    const uint32_t gsize = min(m_tiles - first_m, kGroup);
    const uint32_t in_group = bid % (kGroup * n_tiles);
    const uint32_t tile_m = first_m + in_group % gsize;
    const uint32_t tile_n = in_group / gsize;
    const uint32_t m0 = tile_m * T::BM;
    const uint32_t n0 = tile_n * T::BN;

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
            uint32_t dr = GATHER ? rows[mi] : mi;
            dr = dr < R ? dr : R - 1;
            src[i] = D + (uint64_t)dr * pitch + seg_off[i];
        } else {
            src[i] = reinterpret_cast<const uint8_t*>(QL) +
                     (uint64_t)(n0 + (uint32_t)min(r, T::BN - 1)) * Cp + seg_off[i];
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
#pragma unroll
            for (int i = 0; i < T::B_LOADS; ++i) {
                uint8_t* dst = stage + (lw + 2 * i) * 1024;
                __builtin_amdgcn_global_load_lds((glb_void_t*)(src[i] + k0), (lds_void_t*)dst,
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
        // Each loader wave waits for its own part of tile t (see k_gemm_ring
        // for the counting; only D loads of the last tile can be skipped).
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
                u32x4 v = *reinterpret_cast<const u32x4*>(sa + r * T::BK + 16 * slot_of(r, seg));
                v ^= centre;
                fa[a] = __builtin_bit_cast(i32x4, v);
            }
#pragma unroll
            for (int b = 0; b < T::TN; ++b) {
                const int r = wn * T::TN * 32 + b * 32 + frow;
                fb[b] = *reinterpret_cast<const i32x4*>(sb + r * T::BK + 16 * slot_of(r, seg));
            }
#pragma unroll
            for (int a = 0; a < T::TM; ++a)
#pragma unroll
                for (int b = 0; b < T::TN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb[b], acc[a][b], 0, 0, 0);
        }
    }

    const uint32_t cterm_base = C * kCentreWord;
#pragma unroll
    for (int g = 0; g < T::TN / 4; ++g) {
        const uint32_t bq = (n0 + wn * T::TN * 32) / 4u + 32u * g + (uint32_t)(lane & 31);
        const uint32_t colterm = 128u * (bq < B ? colsum[bq] - cterm_base : 0u);
#pragma unroll
        for (int a = 0; a < T::TM; ++a) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const uint32_t i = m0 + wm * T::TM * 32 + a * 32 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
                if (i < M && bq < B) {
                    const uint32_t r = GATHER ? rows[i] : i;
                    if (r < R) {
                        const uint32_t p0 = (uint32_t)acc[a][4 * g + 0][v];
                        const uint32_t p1 = (uint32_t)acc[a][4 * g + 1][v];
                        const uint32_t p2 = (uint32_t)acc[a][4 * g + 2][v];
                        const uint32_t p3 = (uint32_t)acc[a][4 * g + 3][v];
                        out[(uint64_t)r * o_ldr + (uint64_t)bq * o_ldb] =
                            p0 + (p1 << 8) + (p2 << 16) + (p3 << 24) + colterm + rowterm[r];
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------- dispatch
struct Gemm {
    const pir_db_t* db;
    const uint32_t* rows;   // gathered rows or null
    uint32_t M;             // output rows
    const int8_t* QL;
    uint32_t Cp, B, N;
    const uint32_t* colsum;
    uint32_t* out;
    uint64_t o_ldr, o_ldb;
};

template <class T>
pir_status launch_ring(const Gemm& g, hipStream_t s) {
    const uint32_t n_tiles = (g.N + T::BN - 1) / T::BN;
    const uint32_t m_tiles = (g.M + T::BM - 1) / T::BM;
    const uint64_t blocks = (uint64_t)n_tiles * m_tiles;
    if (blocks > 0x7FFFFFFFull) return PIR_ERR_SHAPE;
    const pir_db_t* db = g.db;
    const uint32_t R = (uint32_t)db->rows, C = (uint32_t)db->cols;
    if (g.rows)
        k_gemm_ring<T, true><<<(uint32_t)blocks, T::THREADS, T::LDS_BYTES, s>>>(
            db->D, db->pitch, R, C, g.rows, g.M, g.QL, g.Cp, g.B, n_tiles, m_tiles, g.colsum,
            db->rowterm, g.out, g.o_ldr, g.o_ldb);
    else
        k_gemm_ring<T, false><<<(uint32_t)blocks, T::THREADS, T::LDS_BYTES, s>>>(
            db->D, db->pitch, R, C, g.rows, g.M, g.QL, g.Cp, g.B, n_tiles, m_tiles, g.colsum,
            db->rowterm, g.out, g.o_ldr, g.o_ldb);
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

template <class T>
pir_status launch_split(const Gemm& g, hipStream_t s) {
    const uint32_t n_tiles = (g.N + T::BN - 1) / T::BN;
    const uint32_t m_tiles = (g.M + T::BM - 1) / T::BM;
    const uint64_t blocks = (uint64_t)n_tiles * m_tiles;
    if (blocks > 0x7FFFFFFFull) return PIR_ERR_SHAPE;
    const pir_db_t* db = g.db;
    const uint32_t R = (uint32_t)db->rows, C = (uint32_t)db->cols;
    if (g.rows)
        k_gemm_split<T, true><<<(uint32_t)blocks, 256, T::LDS_BYTES, s>>>(
            db->D, db->pitch, R, C, g.rows, g.M, g.QL, g.Cp, g.B, n_tiles, m_tiles, g.colsum,
            db->rowterm, g.out, g.o_ldr, g.o_ldb);
    else
        k_gemm_split<T, false><<<(uint32_t)blocks, 256, T::LDS_BYTES, s>>>(
            db->D, db->pitch, R, C, g.rows, g.M, g.QL, g.Cp, g.B, n_tiles, m_tiles, g.colsum,
            db->rowterm, g.out, g.o_ldr, g.o_ldb);
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

template <class T>
pir_status set_split_lds() {
    if (hipFuncSetAttribute((const void*)k_gemm_split<T, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, T::LDS_BYTES) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_gemm_split<T, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, T::LDS_BYTES) != hipSuccess)
        return PIR_ERR_DEVICE;
    return PIR_OK;
}

template <class T>
pir_status set_ring_lds() {
    if (hipFuncSetAttribute((const void*)k_gemm_ring<T, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, T::LDS_BYTES) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_gemm_ring<T, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, T::LDS_BYTES) != hipSuccess)
        return PIR_ERR_DEVICE;
    return PIR_OK;
}

template <class T>
pir_status launch_reg(const Gemm& g, hipStream_t s) {
    const uint32_t n_tiles = (g.N + T::BN - 1) / T::BN;
    const uint32_t m_tiles = (g.M + T::BM - 1) / T::BM;
    const uint64_t blocks = (uint64_t)n_tiles * m_tiles;
    if (blocks > 0x7FFFFFFFull) return PIR_ERR_SHAPE;
    const pir_db_t* db = g.db;
    const uint32_t R = (uint32_t)db->rows, C = (uint32_t)db->cols;
#define PIR_GEMM(VEC, GATHER)                                                                \
    k_gemm<T, VEC, GATHER><<<(uint32_t)blocks, 256, 0, s>>>(db->D, db->pitch, R, C, g.rows, g.M, \
                                                             g.QL, g.Cp, g.B, n_tiles, g.colsum, \
                                                             db->rowterm, g.out, g.o_ldr, g.o_ldb)
    if (db->aligned) {
        if (g.rows) PIR_GEMM(true, true); else PIR_GEMM(true, false);
    } else {
        if (g.rows) PIR_GEMM(false, true); else PIR_GEMM(false, false);
    }
#undef PIR_GEMM
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

// Kernel variants of the batched product.  Ring variants need a 16-byte
// aligned database with C a multiple of 16; 256-wide tiles need N a
// multiple of 256 (batches above 32 queries, padded to 64).
using Ring128x256S6 = Ring<2, 2, 2, 4, 6>;   // 144 KiB LDS
using Ring128x256S4 = Ring<2, 2, 2, 4, 4>;   //  96 KiB
using Ring256x256S4 = Ring<2, 2, 4, 4, 4>;   // 128 KiB, 128x128 per wave
using Ring128x128S8 = Ring<4, 1, 1, 4, 8>;   // 128 KiB
using Ring8w256x256S4 = Ring<4, 2, 2, 4, 4>;  // 8 waves, 128 KiB
using Ring8w256x256S3 = Ring<4, 2, 2, 4, 3>;  // 8 waves,  96 KiB
using Ring8w128x256S6 = Ring<4, 2, 1, 4, 6>;  // 8 waves, 144 KiB
using Ring8w128x256K128S3 = Ring<4, 2, 1, 4, 3, 128>;  // 8 waves, 144 KiB, 128-byte stages
using Ring128x256K128S3 = Ring<2, 2, 2, 4, 3, 128>;    // 144 KiB
using Ring8w256x256K128S2 = Ring<4, 2, 2, 4, 2, 128>;  // 8 waves, 128 KiB
using Ring128x128K128S4 = Ring<4, 1, 1, 4, 4, 128>;    // 128 KiB
using Split128x256A10B4 = Split<2, 2, 2, 4, 10, 4>;   // 80 + 64 KiB
using Split128x256A12B3 = Split<2, 2, 2, 4, 12, 3>;   // 96 + 48 KiB
using Split256x256A5B4 = Split<2, 2, 4, 4, 5, 4>;     // 80 + 64 KiB
using Split128x128A12B6 = Split<4, 1, 1, 4, 12, 6>;   // 96 + 48 KiB
using Reg128x256 = Tile<2, 2, 2, 4, 128>;
using Reg128x128 = Tile<4, 1, 1, 4, 128>;

struct VariantInfo {
    const char* name;
    bool ring;
    uint32_t bn;
    pir_status (*launch)(const Gemm&, hipStream_t);
};

const VariantInfo kVariants[] = {
    {"auto", false, 0, nullptr},
    {"ring_128x256_s6", true, 256, launch_ring<Ring128x256S6>},
    {"ring_128x256_s4", true, 256, launch_ring<Ring128x256S4>},
    {"ring_256x256_s4", true, 256, launch_ring<Ring256x256S4>},
    {"ring_128x128_s8", true, 128, launch_ring<Ring128x128S8>},
    {"reg_128x256", false, 256, launch_reg<Reg128x256>},
    {"reg_128x128", false, 128, launch_reg<Reg128x128>},
    {"split_128x256_a10b4", true, 256, launch_split<Split128x256A10B4>},
    {"split_128x256_a12b3", true, 256, launch_split<Split128x256A12B3>},
    {"split_256x256_a5b4", true, 256, launch_split<Split256x256A5B4>},
    {"split_128x128_a12b6", true, 128, launch_split<Split128x128A12B6>},
    {"ring8w_256x256_s4", true, 256, launch_ring<Ring8w256x256S4>},
    {"ring8w_256x256_s3", true, 256, launch_ring<Ring8w256x256S3>},
    {"ring8w_128x256_s6", true, 256, launch_ring<Ring8w128x256S6>},
    {"ring8w_128x256_k128_s3", true, 256, launch_ring<Ring8w128x256K128S3>},
    {"ring_128x256_k128_s3", true, 256, launch_ring<Ring128x256K128S3>},
    {"ring8w_256x256_k128_s2", true, 256, launch_ring<Ring8w256x256K128S2>},
    {"ring_128x128_k128_s4", true, 128, launch_ring<Ring128x128K128S4>},
};
constexpr uint32_t kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

bool ring_ok(const pir_db_t* db) { return db->aligned && (db->cols % 16 == 0); }

uint32_t padded_batch(uint32_t B) { return B <= 32u ? 32u : (B + 63u) / 64u * 64u; }

bool variant_valid(const pir_db_t* db, uint32_t B, uint32_t v) {
    if (v == 0) return true;
    if (v >= kNumVariants) return false;
    const VariantInfo& vi = kVariants[v];
    if (vi.ring && !ring_ok(db)) return false;
    return (4u * padded_batch(B)) % vi.bn == 0;
}

uint32_t default_variant(const pir_db_t* db, uint32_t B) {
    const bool narrow = padded_batch(B) == 32u;
    if (ring_ok(db)) return narrow ? 4u : 1u;
    return narrow ? 6u : 5u;
}

struct BatchLayout {
    uint32_t Bp, N, Cp;
    size_t ql_bytes, colsum_off, total;
};

BatchLayout batch_layout(const pir_db_t* db, uint32_t B) {
    BatchLayout L;
    // One group of 32 queries uses a 128-wide tile; larger batches are
    // padded to whole 256-wide tiles (64 queries).  Padded queries are zero.
    L.Bp = padded_batch(B);
    L.N = 4u * L.Bp;
    L.Cp = (uint32_t)round_up(db->cols, kKPad);
    L.ql_bytes = round_up((size_t)L.N * L.Cp, kWsAlign);
    L.colsum_off = L.ql_bytes;
    L.total = L.colsum_off + round_up((size_t)L.Bp * 4, kWsAlign);
    return L;
}

}  // namespace

pir_status mfma_init() {
    pir_status st;
    if ((st = set_ring_lds<Ring128x256S6>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring128x256S4>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring256x256S4>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring128x128S8>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring8w256x256S4>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring8w256x256S3>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring8w128x256S6>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring8w128x256K128S3>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring128x256K128S3>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring8w256x256K128S2>()) != PIR_OK) return st;
    if ((st = set_ring_lds<Ring128x128K128S4>()) != PIR_OK) return st;
    if ((st = set_split_lds<Split128x256A10B4>()) != PIR_OK) return st;
    if ((st = set_split_lds<Split128x256A12B3>()) != PIR_OK) return st;
    if ((st = set_split_lds<Split256x256A5B4>()) != PIR_OK) return st;
    return set_split_lds<Split128x128A12B6>();
}

uint32_t mfma_variant_count() { return kNumVariants; }

const char* mfma_variant_name(uint32_t v) { return v < kNumVariants ? kVariants[v].name : nullptr; }

bool mfma_variant_valid(const pir_db_t* db, uint32_t B, uint32_t v) {
    return variant_valid(db, B, v);
}

size_t mfma_workspace_bytes(const pir_db_t* db, uint32_t B) {
    if (B == 0) return 0;
    return batch_layout(db, B).total;
}

pir_status mfma_answer_batch(const pir_db_t* db, const BatchIO& io, uint32_t B,
                             const uint32_t* rows, uint32_t m, void* ws, size_t ws_bytes,
                             hipStream_t s) {
    const BatchLayout L = batch_layout(db, B);
    if (!ws || ws_bytes < L.total || ((uintptr_t)ws % kWsAlign)) return PIR_ERR_WORKSPACE;
    uint8_t* base = static_cast<uint8_t*>(ws);
    int8_t* QL = reinterpret_cast<int8_t*>(base);
    uint32_t* colsum = reinterpret_cast<uint32_t*>(base + L.colsum_off);
    const uint32_t C = (uint32_t)db->cols;

    k_zero_words<<<(L.Bp + 255) / 256, 256, 0, s>>>(colsum, L.Bp);
    PIR_LAUNCH_CHECK();
    dim3 ig(L.Cp / 64, L.Bp / 32);
    if (io.q_ldj == 1)
        k_ingest<true><<<ig, 256, 0, s>>>(io.Q, io.q_ldj, io.q_ldb, C, B, L.Cp, QL, colsum);
    else
        k_ingest<false><<<ig, 256, 0, s>>>(io.Q, io.q_ldj, io.q_ldb, C, B, L.Cp, QL, colsum);
    PIR_LAUNCH_CHECK();

    const uint32_t M = rows ? m : (uint32_t)db->rows;
    if (M == 0) return PIR_OK;
    uint32_t v = db->variant[batch_bucket(B)];
    if (!variant_valid(db, B, v) || v == 0) v = default_variant(db, B);
    const Gemm g{db, rows, M, QL, L.Cp, B, L.N, colsum, io.out, io.o_ldr, io.o_ldb};
    return kVariants[v].launch(g, s);
}
