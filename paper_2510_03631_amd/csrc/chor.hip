// Chor XOR PIR response (the ENS instantiation, Section 5.1; server step of
// Algorithm 3): for each query bit vector q_b over the r database rows,
//
//     out[b] = XOR over rows i with bit i of q_b set of DB[i]
//
// DB rows are b-bit blocks stored as W 32-bit words (row pitch in words);
// query b is packed 32 rows per word, little-endian (bit j of word k selects
// row 32k + j); bits past the last row are ignored.
//
// Boolean XOR has no matrix-core form (the paper makes the same point for
// tensor cores), so this is a VALU / HBM kernel.  Design for gfx950:
// * a workgroup (256 threads) owns a slab of rows and a range of columns; a
//   lane holds 4 consecutive words (16 bytes) of the block for each query it
//   serves, so every row load is a coalesced 16-byte-per-lane read and the
//   accumulators are G x 16 bytes per lane;
// * selector words are loaded once per 32-row block and read with
//   wave-uniform lane reads, so row choices never diverge within a wave;
// * batches of at most 4 queries (k_chor_stream) read only the rows that
//   some query selects (a single query touches half of the database): the
//   selector words of a whole slab are fetched up front, set bits of 64-row
//   pairs of blocks are taken with a wave-uniform bit scan, and up to 32
//   rows per wave are in flight (non-temporal loads); each row is XORed into
//   every query under a mask;
// * larger batches (k_chor_shared) build, per 4 rows, the 16 XOR
//   combinations of the rows in an LDS table and add one table entry per
//   query (method of the Four Russians): one LDS read and XOR per query per
//   4 rows.  The four waves of a workgroup cover one column slice with
//   different query groups and share each table (built once for 4G
//   queries, double-buffered, one barrier per 4 rows);
// * workgroups are numbered slab-major and dealt to XCDs in contiguous
//   ranges, so the query groups of one slab share its rows in L2;
// * slabs combine into the output with atomicXor (XOR is associative and
//   commutative, so the result does not depend on the order); the output is
//   cleared first by a fill kernel.
#include <string.h>

#include "qpir_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr uint32_t kChunkWords = 4 * kThreads;

// Output before accumulation: zero, or a copy of `init` (the OOP response
// starts from its precomputed value A).
__global__ void k_chor_init(uint32_t* __restrict__ p, const uint32_t* __restrict__ init,
                            uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = init ? init[i] : 0u;
}

template <bool VEC>
__device__ inline u32x4 load_words(const uint32_t* row, uint32_t w, uint32_t W) {
    if (VEC) return *reinterpret_cast<const u32x4*>(row + w);   // W % 4 == 0, aligned
    return u32x4{w < W ? row[w] : 0u, w + 1 < W ? row[w + 1] : 0u,
                 w + 2 < W ? row[w + 2] : 0u, w + 3 < W ? row[w + 3] : 0u};
}

template <bool VEC>
__device__ inline u32x4 load_words_nt(const uint32_t* row, uint32_t w, uint32_t W) {
    if (VEC) return __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(row + w));
    return load_words<false>(row, w, W);
}

__device__ inline uint32_t xcd_remap(uint32_t bid, uint32_t nblk) {
    const uint32_t per = nblk / 8u;
    return bid < per * 8u ? (bid % 8u) * per + bid / 8u : bid;
}

// Batches of at most G queries (G <= 4).  Workgroup = one slab of rows
// [r0, r1), all columns in chunks of 1024 words (lane t: words 4t..4t+3).
// One load per lane fetches the selector words of 64 / G consecutive 32-row
// blocks (lane l: query l / (64/G), block l % (64/G)).  Blocks are taken in
// pairs: the OR of the queries' 64-bit masks names the rows to read, up to
// kDepth of them in flight per wave.
constexpr int kDepth = 32;

template <int G, bool VEC>
__global__ __launch_bounds__(kThreads) void k_chor_stream(const uint32_t* __restrict__ DB,
                                                          uint64_t pitch, uint32_t rows,
                                                          uint32_t W,
                                                          const uint32_t* __restrict__ Q,
                                                          uint32_t qwords, uint32_t B,
                                                          uint32_t slab_rows,
                                                          uint32_t* __restrict__ out) {
    constexpr uint32_t kBlocks = 64 / G;
    static_assert(kBlocks % 2 == 0, "blocks are taken in pairs");
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t slab = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t r0 = slab * slab_rows;
    const uint32_t r1 = min(rows, r0 + slab_rows);

    for (uint32_t c0 = 0; c0 < W; c0 += kChunkWords) {
        if (c0 + 256u * (uint32_t)wave >= W) continue;   // no lane of this wave has words here
        const uint32_t w = c0 + 4u * threadIdx.x;
        const bool active = w < W;
        u32x4 acc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = u32x4{0, 0, 0, 0};

        for (uint32_t base = r0; base < r1; base += 32u * kBlocks) {
            uint32_t qv = 0;
            {
                const uint32_t g = (uint32_t)lane / kBlocks;
                const uint32_t rb = base + 32u * ((uint32_t)lane % kBlocks);
                if (g < B && rb < r1) {
                    qv = Q[(uint64_t)g * qwords + rb / 32u];
                    const uint32_t nrow = min(32u, r1 - rb);
                    if (nrow < 32u) qv &= (1u << nrow) - 1u;
                }
            }
            for (uint32_t jb = 0; jb < kBlocks; jb += 2) {
                const uint32_t rblk = base + 32u * jb;
                if (rblk >= r1) break;                    // uniform
                uint64_t sel[G];
                uint64_t any = 0;
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const uint32_t lo = __builtin_amdgcn_readlane(qv, g * (int)kBlocks + (int)jb);
                    const uint32_t hi = __builtin_amdgcn_readlane(qv, g * (int)kBlocks + (int)jb + 1);
                    sel[g] = (uint64_t)lo | ((uint64_t)hi << 32);
                    any |= sel[g];
                }
                while (any) {
                    uint32_t idx[kDepth];
                    u32x4 d[kDepth];
#pragma unroll
                    for (int k = 0; k < kDepth; ++k) {
                        idx[k] = 0;
                        d[k] = u32x4{0, 0, 0, 0};
                        if (any) {                        // uniform
                            idx[k] = (uint32_t)__builtin_ctzll(any);
                            any &= any - 1u;
                            if (active)
                                d[k] = load_words_nt<VEC>(DB + (uint64_t)(rblk + idx[k]) * pitch,
                                                          w, W);
                        }
                    }
#pragma unroll
                    for (int g = 0; g < G; ++g) {
#pragma unroll
                        for (int k = 0; k < kDepth; ++k) {
                            const uint32_t m = 0u - (uint32_t)((sel[g] >> idx[k]) & 1u);
                            acc[g] ^= d[k] & u32x4{m, m, m, m};
                        }
                    }
                }
            }
        }
        if (active) {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if ((uint32_t)g < B) {
                    uint32_t* o = out + (uint64_t)g * W + w;
                    if (acc[g].x) atomicXor(o, acc[g].x);
                    if (w + 1 < W && acc[g].y) atomicXor(o + 1, acc[g].y);
                    if (w + 2 < W && acc[g].z) atomicXor(o + 2, acc[g].z);
                    if (w + 3 < W && acc[g].w) atomicXor(o + 3, acc[g].w);
                }
            }
        }
    }
}

// Larger batches, shared tables.  The four waves of a workgroup cover the
// same 256-word column slice (lane t: words 4t..4t+3) with different groups
// of G queries (4G per workgroup), so each 4-row XOR table is built once for
// all of them: entry e = (hi part: rows 2-3 by e >> 2) xor (lo part: rows
// 0-1 by e & 3); wave w writes entries 4w .. 4w+3 (entry 0 is kept zero).
// Tables are double-buffered in LDS; one barrier per 4-row step (LDS
// counter only, so row loads issued two steps ahead stay in flight) makes a
// step's table visible and, being passed only after every wave finished the
// previous step's lookups, frees the other buffer for the next build.
__device__ inline void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt((0x3F & 0xF) | ((0x3F >> 4) << 14) | (0x7 << 4) | (0x0 << 8));
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

template <int G, bool VEC>
__global__ __launch_bounds__(kThreads) void k_chor_shared(const uint32_t* __restrict__ DB,
                                                          uint64_t pitch, uint32_t rows,
                                                          uint32_t W,
                                                          const uint32_t* __restrict__ Q,
                                                          uint32_t qwords, uint32_t B,
                                                          uint32_t slab_rows, uint32_t n_qg,
                                                          uint32_t n_cs,
                                                          uint32_t* __restrict__ out) {
    __shared__ u32x4 s_tab[2][16][64];            // [buffer][entry][lane], 32 KiB
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // Workgroups of one slab and column slice are consecutive (their query
    // groups read the same rows), slabs outermost.
    const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t qg = bid % n_qg;
    const uint32_t cs = (bid / n_qg) % n_cs;
    const uint32_t slab = bid / (n_qg * n_cs);
    const uint32_t r0 = slab * slab_rows;
    const uint32_t r1 = min(rows, r0 + slab_rows);
    const uint32_t w = cs * 256u + 4u * lane;
    const bool active = w < W;
    const uint32_t qbase = (qg * 4u + (uint32_t)wave) * G;
    const uint32_t nq = qbase < B ? min((uint32_t)G, B - qbase) : 0u;

    if (wave < 2) s_tab[wave][0][lane] = u32x4{0, 0, 0, 0};
    u32x4 acc[G];
#pragma unroll
    for (int g = 0; g < G; ++g) acc[g] = u32x4{0, 0, 0, 0};

    // Rows this wave needs for its entries: 0 and 1 always; 2 for waves 1
    // and 3; 3 for waves 2 and 3.  Plain loads: the query groups of a slab
    // run on one XCD and read the rows from L2 (non-temporal loads sent them
    // to HBM again; 128 queries 0.70 -> 0.68 ms).
    const bool need2 = wave == 1 || wave == 3;
    const bool need3 = wave >= 2;
    auto load_row = [&](uint32_t r) -> u32x4 {
        return (active && r < r1) ? load_words<VEC>(DB + (uint64_t)r * pitch, w, W)
                                  : u32x4{0, 0, 0, 0};
    };
    auto load_step = [&](uint32_t st, u32x4 (&x)[4]) {
        const uint32_t r = r0 + 4u * st;
        x[0] = load_row(r);
        x[1] = load_row(r + 1);
        x[2] = need2 ? load_row(r + 2) : u32x4{0, 0, 0, 0};
        x[3] = need3 ? load_row(r + 3) : u32x4{0, 0, 0, 0};
    };
    // Selector words of the wave's G queries for one 32-row block.
    // * G <= 16: the address is wave-uniform, so these are scalar loads into
    //   SGPRs and the per-lookup table index is scalar arithmetic.  They are
    //   loaded at a block's first step; the step's barrier waits on the same
    //   counter as the LDS writes, so no separate wait is exposed.  Queries
    //   past B read query B-1's word; their sums are never stored.
    // * G = 32 would spill SGPRs: lane g holds query g's word (one vector
    //   load, prefetched a block ahead) and each lookup reads its lane.
    constexpr bool kScalarSel = G <= 16;
    auto load_sel = [&](uint32_t blk, uint32_t (&sel)[G]) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint32_t b = min(qbase + (uint32_t)g, B - 1u);
            sel[g] = 32u * blk < rows ? Q[(uint64_t)b * qwords + blk] : 0u;
        }
    };
    auto load_sel_lane = [&](uint32_t blk) -> uint32_t {
        const uint32_t b = qbase + (uint32_t)lane;
        return ((uint32_t)lane < nq && 32u * blk < rows) ? Q[(uint64_t)b * qwords + blk] : 0u;
    };

    const uint32_t nsteps = r1 > r0 ? (r1 - r0 + 3u) / 4u : 0u;
    u32x4 xa[4], xb[4];
    load_step(0, xa);
    load_step(1, xb);
    uint32_t qv[kScalarSel ? G : 1];
    uint32_t qlane = 0, qlane_next = kScalarSel ? 0u : load_sel_lane(r0 / 32u);

    auto step = [&](uint32_t st, u32x4 (&x)[4]) {
        const int buf = st & 1;
        if (st % 8u == 0) {
            if constexpr (kScalarSel) {
                load_sel(r0 / 32u + st / 8u, qv);
            } else {
                qlane = qlane_next;
                qlane_next = load_sel_lane(r0 / 32u + st / 8u + 1u);
            }
        }
        const u32x4 lo1 = x[0], lo2 = x[1], lo3 = x[0] ^ x[1];
        const u32x4 hi = wave == 0 ? u32x4{0, 0, 0, 0}
                                   : (wave == 1 ? x[2] : (wave == 2 ? x[3] : x[2] ^ x[3]));
        if (wave != 0) s_tab[buf][4 * wave][lane] = hi;
        s_tab[buf][4 * wave + 1][lane] = hi ^ lo1;
        s_tab[buf][4 * wave + 2][lane] = hi ^ lo2;
        s_tab[buf][4 * wave + 3][lane] = hi ^ lo3;
        if (st + 2u < nsteps) load_step(st + 2u, x);    // prefetch two steps ahead
        lds_barrier();
        const int sh = 4 * (int)(st % 8u);
#pragma unroll
        for (int g0 = 0; g0 < G; g0 += 8) {
            u32x4 t[8];
#pragma unroll
            for (int g = 0; g < 8 && g0 + g < G; ++g) {
                const uint32_t word = kScalarSel ? qv[kScalarSel ? g0 + g : 0]
                                                 : __builtin_amdgcn_readlane(qlane, g0 + g);
                const uint32_t idx = (word >> sh) & 15u;
                t[g] = s_tab[buf][idx][lane];
            }
#pragma unroll
            for (int g = 0; g < 8 && g0 + g < G; ++g) acc[g0 + g] ^= t[g];
        }
    };
    for (uint32_t st = 0; st < nsteps; st += 2) {
        step(st, xa);
        if (st + 1 < nsteps) step(st + 1, xb);
    }

    if (active) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if ((uint32_t)g < nq) {
                uint32_t* o = out + (uint64_t)(qbase + g) * W + w;
                if (acc[g].x) atomicXor(o, acc[g].x);
                if (w + 1 < W && acc[g].y) atomicXor(o + 1, acc[g].y);
                if (w + 2 < W && acc[g].z) atomicXor(o + 2, acc[g].z);
                if (w + 3 < W && acc[g].w) atomicXor(o + 3, acc[g].w);
            }
        }
    }
}

// The same with 8-row steps, for groups of 32 queries per wave: two 16-entry
// tables per step (rows 0-3 and rows 4-7 of the step), and each query adds
// one entry of each, acc ^= t0 ^ t1, one three-input XOR per word for two
// lookups.  Per lookup that is two XOR instructions instead of four, and one
// barrier per 8 rows, against twice the table memory (64 KiB per workgroup,
// double-buffered) and twice the rows in flight per step.  (Written with
// the compiler's bitop3 builtin, the kernel needed 458 registers, one wave
// per SIMD, and ran at half the speed; as inline assembly it keeps 234.)
// a ^ b ^ c as one gfx950 three-input bit operation (truth table 0x96).
__device__ inline uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// NW waves of G queries share each step's two tables.  With four waves a
// wave builds four entries of both tables; with eight, four entries of one
// (waves 0-3 the table of rows 0-3, waves 4-7 that of rows 4-7), so the
// build, which every step waits for at its barrier, is spread over twice the
// queries.  Entry e of a table is hi(e >> 2) ^ lo(e & 3), hi and lo the XOR
// combinations of the half's rows 2-3 and 0-1; wave w builds entries
// 4c .. 4c+3 with c = w % 4.  Rows are plain loads: the query groups of a
// slab read them from L2 (non-temporal loads fetched the database 3.8 times
// from HBM per launch at 1024 queries, plain ones 1.5 times).
template <int G, int NW, bool VEC>
__global__ __launch_bounds__(64 * NW) void k_chor_shared8(const uint32_t* __restrict__ DB,
                                                          uint64_t pitch, uint32_t rows,
                                                          uint32_t W,
                                                          const uint32_t* __restrict__ Q,
                                                          uint32_t qwords, uint32_t B,
                                                          uint32_t slab_rows, uint32_t n_qg,
                                                          uint32_t n_cs,
                                                          uint32_t* __restrict__ out) {
    static_assert(NW == 4 || NW == 8, "four or eight waves");
    constexpr int NH = NW == 4 ? 2 : 1;           // table halves a wave builds
    __shared__ u32x4 s_tab[2][2][16][64];         // [buffer][table][entry][lane], 64 KiB
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = wave & 3;                       // hi combination of the wave's entries
    const int h0 = NW == 4 ? 0 : wave >> 2;       // first table half it builds
    const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t qg = bid % n_qg;
    const uint32_t cs = (bid / n_qg) % n_cs;
    const uint32_t slab = bid / (n_qg * n_cs);
    const uint32_t r0 = slab * slab_rows;
    const uint32_t r1 = min(rows, r0 + slab_rows);
    const uint32_t w = cs * 256u + 4u * lane;
    const bool active = w < W;
    const uint32_t qbase = (qg * (uint32_t)NW + (uint32_t)wave) * G;
    const uint32_t nq = qbase < B ? min((uint32_t)G, B - qbase) : 0u;

    if (c == 0) {                                 // entry 0 of the wave's halves
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < NH; ++i) s_tab[b][h0 + i][0][lane] = u32x4{0, 0, 0, 0};
    }
    u32x4 acc[G];
#pragma unroll
    for (int g = 0; g < G; ++g) acc[g] = u32x4{0, 0, 0, 0};

    // Rows of each 4-row half the wave needs: 0 and 1 always; 2 if c & 1;
    // 3 if c & 2.
    const bool need2 = (c & 1) != 0;
    const bool need3 = (c & 2) != 0;
    auto load_row = [&](uint32_t r) -> u32x4 {
        return (active && r < r1) ? load_words<VEC>(DB + (uint64_t)r * pitch, w, W)
                                  : u32x4{0, 0, 0, 0};
    };
    auto load_step = [&](uint32_t st, u32x4 (&x)[4 * NH]) {
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const uint32_t r = r0 + 8u * st + 4u * (uint32_t)(h0 + i);
            x[4 * i + 0] = load_row(r);
            x[4 * i + 1] = load_row(r + 1);
            x[4 * i + 2] = need2 ? load_row(r + 2) : u32x4{0, 0, 0, 0};
            x[4 * i + 3] = need3 ? load_row(r + 3) : u32x4{0, 0, 0, 0};
        }
    };
    // Selector words of the wave's G queries for one 32-row block, one lane
    // per query (scalar selector words would spill SGPRs at 32 queries).
    auto load_sel_lane = [&](uint32_t blk) -> uint32_t {
        const uint32_t b = qbase + (uint32_t)lane;
        return ((uint32_t)lane < nq && 32u * blk < rows) ? Q[(uint64_t)b * qwords + blk] : 0u;
    };

    const uint32_t nsteps = r1 > r0 ? (r1 - r0 + 7u) / 8u : 0u;
    u32x4 xa[4 * NH], xb[4 * NH];
    load_step(0, xa);
    load_step(1, xb);
    uint32_t qlane = 0, qlane_next = load_sel_lane(r0 / 32u);

    auto step = [&](uint32_t st, u32x4 (&x)[4 * NH]) {
        const int buf = st & 1;
        if (st % 4u == 0) {
            qlane = qlane_next;
            qlane_next = load_sel_lane(r0 / 32u + st / 4u + 1u);
        }
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const u32x4 lo1 = x[4 * i], lo2 = x[4 * i + 1], lo3 = lo1 ^ lo2;
            const u32x4 hi = c == 0 ? u32x4{0, 0, 0, 0}
                                    : (c == 1 ? x[4 * i + 2]
                                              : (c == 2 ? x[4 * i + 3]
                                                        : x[4 * i + 2] ^ x[4 * i + 3]));
            if (c != 0) s_tab[buf][h0 + i][4 * c][lane] = hi;
            s_tab[buf][h0 + i][4 * c + 1][lane] = hi ^ lo1;
            s_tab[buf][h0 + i][4 * c + 2][lane] = hi ^ lo2;
            s_tab[buf][h0 + i][4 * c + 3][lane] = hi ^ lo3;
        }
        if (st + 2u < nsteps) load_step(st + 2u, x);    // prefetch two steps ahead
        lds_barrier();
        const int sh = 8 * (int)(st % 4u);
        // Lookups in groups of two queries, software-pipelined: the LDS reads
        // of group j+1 are issued before the XORs of group j, so the XORs
        // overlap the reads' latency (measured at 1024 queries: 3.64 ->
        // 3.35 ms against groups of four read and then XORed).  Two buffers
        // of two queries hold as many registers as one group of four.
        constexpr int PK = 2;
        constexpr int NG = G / PK;
        u32x4 t0[2][PK], t1[2][PK];
        auto lookups = [&](int j, int bsel) {
#pragma unroll
            for (int g = 0; g < PK; ++g) {
                const uint32_t word = __builtin_amdgcn_readlane(qlane, j * PK + g);
                t0[bsel][g] = s_tab[buf][0][(word >> sh) & 15u][lane];
                t1[bsel][g] = s_tab[buf][1][(word >> (sh + 4)) & 15u][lane];
            }
        };
        lookups(0, 0);
#pragma unroll
        for (int j = 0; j < NG; ++j) {
            if (j + 1 < NG) lookups(j + 1, (j + 1) & 1);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int g = 0; g < PK; ++g) {
                u32x4& a = acc[j * PK + g];   // a ^ t0 ^ t1 in one instruction per word
                const u32x4& y0 = t0[j & 1][g];
                const u32x4& y1 = t1[j & 1][g];
                a.x = xor3(a.x, y0.x, y1.x);
                a.y = xor3(a.y, y0.y, y1.y);
                a.z = xor3(a.z, y0.z, y1.z);
                a.w = xor3(a.w, y0.w, y1.w);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    for (uint32_t st = 0; st < nsteps; st += 2) {
        step(st, xa);
        if (st + 1 < nsteps) step(st + 1, xb);
    }

    if (active) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if ((uint32_t)g < nq) {
                uint32_t* o = out + (uint64_t)(qbase + g) * W + w;
                if (acc[g].x) atomicXor(o, acc[g].x);
                if (w + 1 < W && acc[g].y) atomicXor(o + 1, acc[g].y);
                if (w + 2 < W && acc[g].z) atomicXor(o + 2, acc[g].z);
                if (w + 3 < W && acc[g].w) atomicXor(o + 3, acc[g].w);
            }
        }
    }
}

// NW8 = 0: the 4-row kernel (four waves); 4 or 8: the 8-row kernel with
// that many waves per workgroup.
template <int G, int NW8 = 0>
pir_status launch_shared(const uint32_t* d_DB, uint32_t rows, uint32_t words, uint64_t pitch,
                         const uint32_t* d_Q, uint32_t B, uint32_t* d_out, uint32_t target,
                         hipStream_t s) {
    constexpr int NW = NW8 ? NW8 : 4;
    const uint32_t qwords = (rows + 31) / 32;
    const uint32_t n_qg = (B + NW * G - 1) / (NW * G);
    const uint32_t n_cs = (words + 255) / 256;
    const uint64_t per_slab = (uint64_t)n_qg * n_cs;
    uint64_t n_slabs = target / per_slab;
    if (n_slabs < 1) n_slabs = 1;
    uint64_t slab = (rows + n_slabs - 1) / n_slabs;
    slab = (slab + 31) / 32 * 32;
    if (slab < 32) slab = 32;
    n_slabs = (rows + slab - 1) / slab;
    const uint64_t blocks = n_slabs * per_slab;
    if (blocks > 0x7FFFFFFFull) return PIR_ERR_SHAPE;
    const bool vec = ((uintptr_t)d_DB % 16 == 0) && (words % 4 == 0) && (pitch % 4 == 0);
    if constexpr (NW8 != 0) {
        if (vec)
            k_chor_shared8<G, NW, true><<<(uint32_t)blocks, 64 * NW, 0, s>>>(
                d_DB, pitch, rows, words, d_Q, qwords, B, (uint32_t)slab, n_qg, n_cs, d_out);
        else
            k_chor_shared8<G, NW, false><<<(uint32_t)blocks, 64 * NW, 0, s>>>(
                d_DB, pitch, rows, words, d_Q, qwords, B, (uint32_t)slab, n_qg, n_cs, d_out);
    } else if (vec) {
        k_chor_shared<G, true><<<(uint32_t)blocks, kThreads, 0, s>>>(
            d_DB, pitch, rows, words, d_Q, qwords, B, (uint32_t)slab, n_qg, n_cs, d_out);
    } else {
        k_chor_shared<G, false><<<(uint32_t)blocks, kThreads, 0, s>>>(
            d_DB, pitch, rows, words, d_Q, qwords, B, (uint32_t)slab, n_qg, n_cs, d_out);
    }
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

template <int G>
pir_status launch_stream(const uint32_t* d_DB, uint32_t rows, uint32_t words, uint64_t pitch,
                         const uint32_t* d_Q, uint32_t B, uint32_t* d_out, hipStream_t s) {
    const uint32_t qwords = (rows + 31) / 32;
    // Enough rows in flight to stream HBM (32 per wave), few enough slabs to
    // keep the output atomics (slabs x B x words, all onto the same B rows
    // of words) down: at most one workgroup per CU for a single query, two
    // for more, and at least 256 rows per slab.  (Measured on 2^18 and 2^16
    // rows of 3 KB: fewer workgroups starve the stream on the large
    // database, more slabs spend the small one's time in atomics.)
    const uint32_t target = G == 1 ? 256u : 512u;
    uint64_t slab = (rows + target - 1) / target;
    slab = (slab + 31) / 32 * 32;
    if (slab < 256) slab = 256;
    const uint64_t blocks = (rows + slab - 1) / slab;
    if (blocks > 0x7FFFFFFFull) return PIR_ERR_SHAPE;
    const bool vec = ((uintptr_t)d_DB % 16 == 0) && (words % 4 == 0) && (pitch % 4 == 0);
    if (vec)
        k_chor_stream<G, true><<<(uint32_t)blocks, kThreads, 0, s>>>(d_DB, pitch, rows, words, d_Q,
                                                                     qwords, B, (uint32_t)slab,
                                                                     d_out);
    else
        k_chor_stream<G, false><<<(uint32_t)blocks, kThreads, 0, s>>>(d_DB, pitch, rows, words, d_Q,
                                                                      qwords, B, (uint32_t)slab,
                                                                      d_out);
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

}  // namespace

bool current_is_gfx950() {
    int dev = -1;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return false;
    return strncmp(prop.gcnArchName, "gfx950", 6) == 0;
}

pir_status chor_init(uint32_t* d_out, const uint32_t* d_init, uint64_t n, hipStream_t s) {
    if (n == 0) return PIR_OK;
    if ((n + 255) / 256 > 0x7FFFFFFFull) return PIR_ERR_SHAPE;
    k_chor_init<<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(d_out, d_init, n);
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

pir_status chor_xor(const uint32_t* d_DB, uint32_t rows, uint32_t words, uint64_t pitch,
                    const uint32_t* d_Q, uint32_t B, const uint32_t* d_init, uint32_t* d_out,
                    hipStream_t s) {
    const pir_status st = chor_init(d_out, d_init, (uint64_t)B * words, s);
    if (st != PIR_OK) return st;
    // Small batches stream every row under masks; larger ones use the
    // XOR tables.  Fewer, longer slabs for large batches keep the number of
    // output atomics down.
    if (B == 1) return launch_stream<1>(d_DB, rows, words, pitch, d_Q, B, d_out, s);
    if (B <= 4) return launch_stream<4>(d_DB, rows, words, pitch, d_Q, B, d_out, s);
    if (B <= 16) return launch_shared<4>(d_DB, rows, words, pitch, d_Q, B, d_out, 768, s);
    if (B <= 32) return launch_shared<8>(d_DB, rows, words, pitch, d_Q, B, d_out, 1024, s);
    if (B <= 256) {
        // Groups of 16: the 8-row kernel with eight waves (128 queries per
        // table) when that pads the batch no further than the 4-row
        // kernel's 64 per workgroup and its slabs keep at least 1024 rows;
        // shorter slabs spend the time in their output atomics.  Measured
        // on 2^18 rows of 3 KB: 128 queries 680 -> 654 us, 200 1155 ->
        // 1017 us, 256 1188 -> 1086 us; 64 stays with the 4-row kernel (400
        // against 543 us), and so does the CIP-PIR flip chunk of 2^16 rows
        // (128 queries 246 against 335 us, 256 362 against 428 us).
        const uint32_t pad64 = (B + 63) / 64 * 64, pad128 = (B + 127) / 128 * 128;
        const uint64_t per_slab8 = (uint64_t)(pad128 / 128) * ((words + 255) / 256);
        const uint64_t slabs8 = per_slab8 >= 768 ? 1 : 768 / per_slab8;
        if (pad128 <= pad64 && rows / slabs8 >= 1024)
            return launch_shared<16, 8>(d_DB, rows, words, pitch, d_Q, B, d_out, 768, s);
        return launch_shared<16>(d_DB, rows, words, pitch, d_Q, B, d_out, 768, s);
    }
    // Above 256: the 8-row kernel.  Eight waves per workgroup (one per CU)
    // share each table across 256 queries, which halves the table build per
    // query, but pad the batch to a multiple of 256; four waves (two
    // workgroups per CU) pad to 128.  Eight when that pads no further
    // (measured: 1024 queries 3.33 -> 2.91 ms, 512 1.76 -> 1.60 ms; 300
    // stays with four, 1.33 against 1.47 ms).
    const uint32_t pad4 = (B + 127) / 128 * 128, pad8 = (B + 255) / 256 * 256;
    if (pad8 <= pad4) return launch_shared<32, 8>(d_DB, rows, words, pitch, d_Q, B, d_out, 256, s);
    return launch_shared<32, 4>(d_DB, rows, words, pitch, d_Q, B, d_out, 512, s);
}

extern "C" {

pir_status pir_chor_answer(const uint32_t* d_DB, uint32_t rows, uint32_t words,
                           uint64_t row_pitch_words, const uint32_t* d_Q, uint32_t B,
                           uint32_t* d_out, pir_stream_t stream) {
    if (B == 0) return PIR_OK;
    if (!d_DB || !d_Q || !d_out) return PIR_ERR_INVALID_ARG;
    if (rows == 0 || words == 0 || row_pitch_words < words || rows > kMaxDim ||
        words > kMaxDim || B > kMaxBatch)
        return PIR_ERR_SHAPE;
    if (!current_is_gfx950()) return PIR_ERR_UNSUPPORTED;
    return chor_xor(d_DB, rows, words, row_pitch_words, d_Q, B, nullptr, d_out,
                    static_cast<hipStream_t>(stream));
}

}  // extern "C"
