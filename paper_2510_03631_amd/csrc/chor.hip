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
// * a workgroup (256 threads) owns a slab of rows, a group of up to G = 16
//   queries and a 1024-word column chunk: lane t holds words 4t..4t+3 of the
//   chunk for every query of the group (G x 16-byte accumulators);
// * per 32-row block the group's selector words are loaded once (lane g
//   holds query g's word; wave-uniform reads pick bits out), and rows are
//   loaded 8 at a time, back to back;
// * batches of at most 4 queries (k_chor_stream) read only the rows that
//   some query selects (a single query touches half of the database): the
//   selector words of a whole slab are fetched up front, set bits of 64-row
//   pairs of blocks are taken with a wave-uniform bit scan, and up to 32
//   rows per wave are in flight (non-temporal loads); each row is XORed into
//   every query under a mask;
// * larger batches (k_chor) build, per 4 rows, the 16 XOR combinations of
//   the rows in a wave-private LDS table and add one table entry per query
//   (method of the Four Russians): one LDS read and XOR per query per 4 rows;
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

// Work of one workgroup: rows [r0, r1) of a slab, queries [b0, b0 + nb) of a
// group, all columns in chunks of 1024 words (lane t: words 4t..4t+3).
//
// TABLE == false (batches of at most 4): every row is streamed and XORed
// under a wave-uniform mask, acc_g ^= row & -(bit), no branches.
// TABLE == true: for every 4 consecutive rows the wave writes the 16 XOR
// combinations of its slice into a private LDS table (method of the Four
// Russians); each query then costs one LDS read at the index given by its
// 4 selector bits and one XOR, instead of a test and XOR per row.
template <int G, bool TABLE, bool VEC>
__global__ __launch_bounds__(kThreads) void k_chor(const uint32_t* __restrict__ DB, uint64_t pitch,
                                                   uint32_t rows, uint32_t W,
                                                   const uint32_t* __restrict__ Q, uint32_t qwords,
                                                   uint32_t B, uint32_t slab_rows,
                                                   uint32_t n_groups, uint32_t* __restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) u32x4 s_table[];   // [wave][16][64]
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    u32x4* tab = s_table + wave * 16 * 64;

    uint32_t bid = blockIdx.x;
    {
        const uint32_t per = gridDim.x / 8u;
        if (bid < per * 8u) bid = (bid % 8u) * per + bid / 8u;
    }
    const uint32_t slab = bid / n_groups;
    const uint32_t grp = bid % n_groups;
    const uint32_t r0 = slab * slab_rows;
    const uint32_t r1 = min(rows, r0 + slab_rows);
    const uint32_t b0 = grp * G;
    const uint32_t nb = min((uint32_t)G, B - b0);
    if (TABLE) tab[lane] = u32x4{0, 0, 0, 0};   // entry 0: no row selected

    for (uint32_t c0 = 0; c0 < W; c0 += kChunkWords) {
        // A wave whose 64 lanes all lie past the last word has nothing to do
        // in this chunk (3 KB blocks leave the fourth wave idle); the waves
        // never synchronize with each other, so it moves on.
        if (c0 + 256u * (uint32_t)wave >= W) continue;
        const uint32_t w = c0 + 4u * threadIdx.x;
        const bool active = w < W;
        u32x4 acc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = u32x4{0, 0, 0, 0};

        for (uint32_t r = r0; r < r1; r += 32) {
            const uint32_t nrow = min(32u, r1 - r);
            const uint32_t valid = nrow == 32 ? 0xFFFFFFFFu : ((1u << nrow) - 1u);
            // Lane g < nb holds query g's 32 selector bits for this block.
            const uint32_t qv = (uint32_t)lane < nb ? (Q[(uint64_t)(b0 + lane) * qwords + r / 32] & valid)
                                                    : 0u;
#pragma unroll 1
            for (int s8 = 0; s8 < 32; s8 += 8) {
                u32x4 d[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    d[k] = u32x4{0, 0, 0, 0};
                    if ((uint32_t)(s8 + k) < nrow && active)
                        d[k] = load_words<VEC>(DB + (uint64_t)(r + s8 + k) * pitch, w, W);
                }
                if (!TABLE) {
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const uint32_t q = __builtin_amdgcn_readlane(qv, g);
#pragma unroll
                        for (int k = 0; k < 8; ++k) {
                            const uint32_t m = 0u - ((q >> (s8 + k)) & 1u);
                            acc[g] ^= d[k] & u32x4{m, m, m, m};
                        }
                    }
                } else {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const u32x4 x0 = d[4 * h], x1 = d[4 * h + 1], x2 = d[4 * h + 2],
                                    x3 = d[4 * h + 3];
                        const u32x4 t3 = x0 ^ x1, t5 = x2 ^ x0, t6 = x2 ^ x1, t7 = x2 ^ t3;
                        // Entries 1..15 (entry i XORs the rows whose bit is set in i).
                        tab[1 * 64 + lane] = x0;
                        tab[2 * 64 + lane] = x1;
                        tab[3 * 64 + lane] = t3;
                        tab[4 * 64 + lane] = x2;
                        tab[5 * 64 + lane] = t5;
                        tab[6 * 64 + lane] = t6;
                        tab[7 * 64 + lane] = t7;
                        tab[8 * 64 + lane] = x3;
                        tab[9 * 64 + lane] = x3 ^ x0;
                        tab[10 * 64 + lane] = x3 ^ x1;
                        tab[11 * 64 + lane] = x3 ^ t3;
                        tab[12 * 64 + lane] = x3 ^ x2;
                        tab[13 * 64 + lane] = x3 ^ t5;
                        tab[14 * 64 + lane] = x3 ^ t6;
                        tab[15 * 64 + lane] = x3 ^ t7;
                        // Each lane reads only its own column of the table
                        // (entry * 64 + lane), so the table is per-lane data:
                        // program order alone orders these reads after the
                        // writes above and before the next writes.
                        // Lookups in batches of 8: the reads are issued together
                        // so that several are in flight before the XORs wait.
                        const int sh = s8 + 4 * h;
#pragma unroll
                        for (int g0 = 0; g0 < G; g0 += 8) {
                            u32x4 t[8];
#pragma unroll
                            for (int g = 0; g < 8; ++g) {
                                const uint32_t idx =
                                    (__builtin_amdgcn_readlane(qv, g0 + g) >> sh) & 15u;
                                t[g] = tab[idx * 64 + lane];
                            }
#pragma unroll
                            for (int g = 0; g < 8; ++g) acc[g0 + g] ^= t[g];
                        }
                    }
                }
                if ((uint32_t)(s8 + 8) >= nrow) break;
            }
        }
        if (active) {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if ((uint32_t)g < nb) {
                    uint32_t* o = out + (uint64_t)(b0 + g) * W + w;
                    if (acc[g].x) atomicXor(o, acc[g].x);
                    if (w + 1 < W && acc[g].y) atomicXor(o + 1, acc[g].y);
                    if (w + 2 < W && acc[g].z) atomicXor(o + 2, acc[g].z);
                    if (w + 3 < W && acc[g].w) atomicXor(o + 3, acc[g].w);
                }
            }
        }
    }
}

template <int G, bool TABLE>
pir_status launch_chor(const uint32_t* d_DB, uint32_t rows, uint32_t words, uint64_t pitch,
                       const uint32_t* d_Q, uint32_t B, uint32_t* d_out, uint32_t target_blocks,
                       hipStream_t s) {
    const uint32_t qwords = (rows + 31) / 32;
    const uint32_t n_groups = (B + G - 1) / G;
    uint64_t slab = ((uint64_t)rows * n_groups + target_blocks - 1) / target_blocks;
    slab = (slab + 31) / 32 * 32;
    if (slab < 32) slab = 32;
    const uint64_t n_slabs = (rows + slab - 1) / slab;
    const uint64_t blocks = n_slabs * n_groups;
    if (blocks > 0x7FFFFFFFull) return PIR_ERR_SHAPE;
    const size_t lds = TABLE ? (size_t)4 * 16 * 64 * sizeof(u32x4) : 0;
    const bool vec = ((uintptr_t)d_DB % 16 == 0) && (words % 4 == 0) && (pitch % 4 == 0);
    if (vec)
        k_chor<G, TABLE, true><<<(uint32_t)blocks, kThreads, lds, s>>>(
            d_DB, pitch, rows, words, d_Q, qwords, B, (uint32_t)slab, n_groups, d_out);
    else
        k_chor<G, TABLE, false><<<(uint32_t)blocks, kThreads, lds, s>>>(
            d_DB, pitch, rows, words, d_Q, qwords, B, (uint32_t)slab, n_groups, d_out);
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
    // 4-row tables.  Fewer, longer slabs for large batches keep the number of
    // output atomics down.
    if (B == 1) return launch_stream<1>(d_DB, rows, words, pitch, d_Q, B, d_out, s);
    if (B <= 4) return launch_stream<4>(d_DB, rows, words, pitch, d_Q, B, d_out, s);
    if (B <= 64) return launch_chor<16, true>(d_DB, rows, words, pitch, d_Q, B, d_out, 512, s);
    return launch_chor<32, true>(d_DB, rows, words, pitch, d_Q, B, d_out, 512, s);
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
