// Single-query Answer: a[r] = sum_j D[r][j] * q[j] mod 2^32.
//
// The server's per-query response (Definition 1) is a matrix-vector product
// whose cost is streaming the database once: every byte of D is used once,
// so the kernel is bound by HBM bandwidth (the paper makes the same
// observation for its XOR variant in Section 5.2: low operational intensity,
// coalescing rather than matrix units).  Design for gfx950:
//
// * q is split into four byte limbs, q = sum_k 2^(8k) q_k, so that
//   a = sum_k 2^(8k) (D q_k).  Each D q_k is a sum of byte x byte products,
//   one v_dot4_u32_u8 per four database bytes and limb, plus a shift-add
//   per limb every 16 bytes: ~1.25 VALU lane-ops per database byte, far
//   under the ~4.9 the CUs can spend at full HBM rate.  All arithmetic
//   wraps modulo 2^32, which is all the answer needs.
// * A workgroup (4 waves) stages a slice of kSlice query words in LDS as the
//   four limb planes (split once per workgroup, not per wave).
// * Each wave owns RW database rows.  One wave-wide 16-byte load covers 1024
//   contiguous bytes of a row (fully coalesced); the RW row loads of a chunk
//   are issued back to back so RW KiB per wave are in flight.  The stream is
//   read with non-temporal loads.
// * After the column loop each lane holds RW partial sums; they are
//   transposed through LDS and finished with lane shuffles, so one lane per
//   row writes the result.
// * Shapes with too few row blocks to fill the chip split the columns; the
//   per-split partial sums go to the workspace and a second kernel adds
//   them (integer addition modulo 2^32 is exact in any order).
#include <type_traits>

#include "qpir_internal.h"

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kChunk = 1024;   // columns covered by one wave-wide 16-byte load
constexpr int kSlice = 4096;   // query words staged in LDS at a time
constexpr int kRW = 16;        // rows per wave of the default variant

// Four consecutive query words -> the four limb words; limb k holds byte k
// of each word, the first word in the low byte.
__device__ inline void limbs_of4(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                 uint32_t out[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int sh = 8 * k;
        out[k] = ((x0 >> sh) & 0xFFu) | (((x1 >> sh) & 0xFFu) << 8) |
                 (((x2 >> sh) & 0xFFu) << 16) | (((x3 >> sh) & 0xFFu) << 24);
    }
}

// 16 bytes of a row starting at column c, zero past column `end`.
template <bool VEC>
__device__ inline u32x4 load16(const uint8_t* row, uint32_t c, uint32_t end) {
    if (VEC && c + 16 <= end) {
        return __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(row + c));
    }
    uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const uint32_t b = (c + e < end) ? row[c + e] : 0u;
        w[e >> 2] |= b << (8 * (e & 3));
    }
    return u32x4{w[0], w[1], w[2], w[3]};
}

// 16 database bytes times the matching 16 query words, mod 2^32: per limb k
// a chain of four dot4 products (at most 16 * 255 * 255 < 2^21, exact), then
// sum_k 2^(8k) p_k.  Combining per chunk keeps one accumulator per row.
__device__ inline uint32_t dot16(const u32x4 d, const u32x4 L[4]) {
    uint32_t p[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t a = __builtin_amdgcn_udot4(d.x, L[k].x, 0u, false);
        a = __builtin_amdgcn_udot4(d.y, L[k].y, a, false);
        a = __builtin_amdgcn_udot4(d.z, L[k].z, a, false);
        p[k] = __builtin_amdgcn_udot4(d.w, L[k].w, a, false);
    }
    return p[0] + (p[1] << 8) + (p[2] << 16) + (p[3] << 24);
}

template <int RW, bool VEC>
__global__ __launch_bounds__(kThreads) void k_answer1(const uint8_t* __restrict__ D, uint64_t pitch,
                                                      uint32_t R, uint32_t C,
                                                      const uint32_t* __restrict__ q,
                                                      uint32_t* __restrict__ out,
                                                      uint32_t cols_per_split) {
    __shared__ u32x4 s_limb[4][kSlice / 16];
    __shared__ uint32_t s_red[kWaves][RW][65];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // Wave-uniform, so the row addresses live in scalar registers.
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint32_t row0 = (blockIdx.x * kWaves + wave) * RW;
    const uint32_t cb = blockIdx.y * cols_per_split;
    const uint32_t ce = min(C, cb + cols_per_split);

    // Rows past the end re-read the last row; their sums are never stored.
    const uint8_t* rp[RW];
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const uint32_t r = min(row0 + (uint32_t)i, R - 1);
        rp[i] = D + (uint64_t)r * pitch;
    }

    uint32_t acc[RW];
#pragma unroll
    for (int i = 0; i < RW; ++i) acc[i] = 0;

    for (uint32_t s0 = cb; s0 < ce; s0 += kSlice) {
        const uint32_t se = min(ce, s0 + (uint32_t)kSlice);
        __syncthreads();   // previous slice fully consumed
        for (int t = tid; t < kSlice / 16; t += kThreads) {
            const uint32_t c = s0 + 16u * t;
            uint32_t x[16];
            if (VEC && c + 16 <= se) {
                const u32x4* qp = reinterpret_cast<const u32x4*>(q + c);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const u32x4 w = qp[v];
                    x[4 * v + 0] = w.x;
                    x[4 * v + 1] = w.y;
                    x[4 * v + 2] = w.z;
                    x[4 * v + 3] = w.w;
                }
            } else {
#pragma unroll
                for (int e = 0; e < 16; ++e) x[e] = (c + e < se) ? q[c + e] : 0u;
            }
            uint32_t l[4][4];
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                uint32_t o[4];
                limbs_of4(x[4 * w], x[4 * w + 1], x[4 * w + 2], x[4 * w + 3], o);
#pragma unroll
                for (int k = 0; k < 4; ++k) l[k][w] = o[k];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) s_limb[k][t] = u32x4{l[k][0], l[k][1], l[k][2], l[k][3]};
        }
        __syncthreads();

        for (uint32_t c0 = s0; c0 < se; c0 += kChunk) {
            const uint32_t li = (c0 - s0) / 16 + lane;
            u32x4 L[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) L[k] = s_limb[k][li];
            const uint32_t c = c0 + 16u * lane;
            if (VEC && c0 + kChunk <= se) {
                u32x4 d[RW];
#pragma unroll
                for (int i = 0; i < RW; ++i)
                    d[i] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(rp[i] + c));
#pragma unroll
                for (int i = 0; i < RW; ++i) acc[i] += dot16(d[i], L);
            } else if (c < se) {
#pragma unroll
                for (int i = 0; i < RW; ++i) acc[i] += dot16(load16<VEC>(rp[i], c, se), L);
            }
        }
    }

    // Sum the 64 lanes of each row.
#pragma unroll
    for (int i = 0; i < RW; ++i) s_red[wave][i][lane] = acc[i];
    __syncthreads();
    constexpr int kLanesPerRow = 64 / RW;
    const int i = lane / kLanesPerRow;
    const int part = lane % kLanesPerRow;
    uint32_t v = 0;
#pragma unroll
    for (int t = 0; t < RW; ++t) v += s_red[wave][i][part * RW + t];
#pragma unroll
    for (int off = 1; off < kLanesPerRow; off <<= 1) v += __shfl_xor(v, off);
    const uint32_t r = row0 + (uint32_t)i;
    if (part == 0 && r < R) out[(uint64_t)blockIdx.y * R + r] = v;
}

__global__ void k_sum_splits(const uint32_t* __restrict__ part, uint32_t R, uint32_t S,
                             uint32_t* __restrict__ out) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    uint32_t v = 0;
    for (uint32_t s = 0; s < S; ++s) v += part[(uint64_t)s * R + r];
    out[r] = v;
}

struct SplitPlan {
    uint32_t splits;
    uint32_t cols_per_split;
};

// Split the columns only when the row blocks alone cannot give every CU
// a workgroup; then aim at about four workgroups per CU, so the last
// round's stragglers stay short (measured on the 3072 x 2^18 field-form
// database, 48 row blocks: 11 splits 147 us, 21-32 splits 137-139 us).
SplitPlan plan_splits(const pir_db_t* db, uint32_t rows_per_block) {
    const uint64_t blocks = (db->rows + rows_per_block - 1) / rows_per_block;
    const uint64_t chunks = (db->cols + kChunk - 1) / kChunk;
    uint64_t s = 1;
    if (blocks < 256) s = (1024 + blocks - 1) / blocks;
    if (s > chunks) s = chunks;
    if (s < 1) s = 1;
    uint64_t cps = ((db->cols + s - 1) / s + kChunk - 1) / kChunk * kChunk;
    s = (db->cols + cps - 1) / cps;
    return SplitPlan{(uint32_t)s, (uint32_t)cps};
}

size_t split_bytes(const pir_db_t* db, uint32_t rows_per_block) {
    const SplitPlan p = plan_splits(db, rows_per_block);
    return p.splits > 1 ? round_up((size_t)p.splits * db->rows * 4, kWsAlign) : 0;
}

template <int RW>
pir_status launch_answer1(const pir_db_t* db, const uint32_t* q, uint32_t* a, void* ws,
                          size_t ws_bytes, hipStream_t s) {
    constexpr uint32_t kRows = RW * kWaves;
    const SplitPlan p = plan_splits(db, kRows);
    const uint32_t R = (uint32_t)db->rows, C = (uint32_t)db->cols;
    uint32_t* dst = a;
    if (p.splits > 1) {
        if (!ws || ws_bytes < split_bytes(db, kRows) || ((uintptr_t)ws % kWsAlign))
            return PIR_ERR_WORKSPACE;
        dst = static_cast<uint32_t*>(ws);
    }
    const bool vec = db->aligned && ((uintptr_t)q % 16 == 0);
    dim3 grid((R + kRows - 1) / kRows, p.splits);
    if (vec)
        k_answer1<RW, true><<<grid, kThreads, 0, s>>>(db->D, db->pitch, R, C, q, dst,
                                                      p.cols_per_split);
    else
        k_answer1<RW, false><<<grid, kThreads, 0, s>>>(db->D, db->pitch, R, C, q, dst,
                                                       p.cols_per_split);
    PIR_LAUNCH_CHECK();
    if (p.splits > 1) {
        k_sum_splits<<<(R + 255) / 256, 256, 0, s>>>(dst, R, p.splits, a);
        PIR_LAUNCH_CHECK();
    }
    return PIR_OK;
}

struct GemvVariant {
    const char* name;
    uint32_t rows_per_wave;
    pir_status (*launch)(const pir_db_t*, const uint32_t*, uint32_t*, void*, size_t, hipStream_t);
};

const GemvVariant kGemv[] = {
    {"auto", kRW, launch_answer1<kRW>},
    {"rows16", 16, launch_answer1<16>},
    {"rows8", 8, launch_answer1<8>},
    {"rows32", 32, launch_answer1<32>},
};
constexpr uint32_t kNumGemv = sizeof(kGemv) / sizeof(kGemv[0]);

// ---------------------------------------------------------------- few queries
// Batches of at most 4 queries (and the field form's single query): the same
// stream over D as k_answer1, with the limb planes of NQ queries staged in
// LDS and NQ accumulators per row, so D is read once for the whole batch.
// On the matrix cores a batch is padded to 32 queries (128 limb rows), so
// for NQ <= 4 this stream is the faster route: per 16 database bytes and
// query it costs 16 dot4 plus a combine, 1.2 VALU lane-ops per byte and
// query against the ~4.9 the CUs can spend at full HBM rate.
//
// EXACT (field form): each chunk's combined limb products are below 2^45
// (four dot4 chains of at most 16 * 255 * 255 < 2^21, shifted by 8k) and are
// added into 64-bit accumulators; D q < 2^63 for C <= 2^23, so the sum is
// the exact integer, reduced mod p once at the end.
constexpr int kFewSlice = 2048;   // query words per LDS stage

template <int NQ, int RW, bool VEC, bool EXACT>
__global__ __launch_bounds__(kThreads) void k_answer_few(
    const uint8_t* __restrict__ D, uint64_t pitch, uint32_t R, uint32_t C,
    const uint32_t* __restrict__ Q, uint64_t ldj, uint64_t ldb, uint32_t B,
    uint32_t cols_per_split, void* __restrict__ part) {
    typedef typename std::conditional<EXACT, uint64_t, uint32_t>::type acc_t;
    __shared__ u32x4 s_limb[NQ][4][kFewSlice / 16];
    __shared__ acc_t s_red[kWaves][RW][65];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint32_t row0 = (blockIdx.x * kWaves + wave) * RW;
    const uint32_t cb = blockIdx.y * cols_per_split;
    const uint32_t ce = min(C, cb + cols_per_split);

    const uint8_t* rp[RW];
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const uint32_t r = min(row0 + (uint32_t)i, R - 1);
        rp[i] = D + (uint64_t)r * pitch;
    }
    acc_t acc[RW][NQ];
#pragma unroll
    for (int i = 0; i < RW; ++i)
#pragma unroll
        for (int b = 0; b < NQ; ++b) acc[i][b] = 0;

    for (uint32_t s0 = cb; s0 < ce; s0 += kFewSlice) {
        const uint32_t se = min(ce, s0 + (uint32_t)kFewSlice);
        __syncthreads();   // previous slice fully consumed
        for (int t = tid; t < NQ * (kFewSlice / 16); t += kThreads) {
            const int b = t / (kFewSlice / 16);
            const int g = t % (kFewSlice / 16);
            const uint32_t c = s0 + 16u * g;
            uint32_t x[16];
#pragma unroll
            for (int e = 0; e < 16; ++e)
                x[e] = ((uint32_t)b < B && c + e < se) ? Q[(uint64_t)(c + e) * ldj + (uint64_t)b * ldb]
                                                       : 0u;
            uint32_t l[4][4];
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                uint32_t o[4];
                limbs_of4(x[4 * w], x[4 * w + 1], x[4 * w + 2], x[4 * w + 3], o);
#pragma unroll
                for (int k = 0; k < 4; ++k) l[k][w] = o[k];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) s_limb[b][k][g] = u32x4{l[k][0], l[k][1], l[k][2], l[k][3]};
        }
        __syncthreads();

        for (uint32_t c0 = s0; c0 < se; c0 += kChunk) {
            const uint32_t li = (c0 - s0) / 16 + lane;
            const uint32_t c = c0 + 16u * lane;
            u32x4 d[RW];
            if (VEC && c0 + kChunk <= se) {
#pragma unroll
                for (int i = 0; i < RW; ++i)
                    d[i] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(rp[i] + c));
            } else {
#pragma unroll
                for (int i = 0; i < RW; ++i) d[i] = c < se ? load16<VEC>(rp[i], c, se) : u32x4{0, 0, 0, 0};
            }
#pragma unroll
            for (int b = 0; b < NQ; ++b) {
                u32x4 L[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) L[k] = s_limb[b][k][li < kFewSlice / 16 ? li : 0];
#pragma unroll
                for (int i = 0; i < RW; ++i) {
                    if (EXACT) {
                        uint32_t p[4];
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            uint32_t a = __builtin_amdgcn_udot4(d[i].x, L[k].x, 0u, false);
                            a = __builtin_amdgcn_udot4(d[i].y, L[k].y, a, false);
                            a = __builtin_amdgcn_udot4(d[i].z, L[k].z, a, false);
                            p[k] = __builtin_amdgcn_udot4(d[i].w, L[k].w, a, false);
                        }
                        acc[i][b] += (uint64_t)p[0] + ((uint64_t)p[1] << 8) +
                                     ((uint64_t)p[2] << 16) + ((uint64_t)p[3] << 24);
                    } else {
                        acc[i][b] += dot16(d[i], L);
                    }
                }
            }
        }
    }

    // Sum the 64 lanes of each (row, query); one query at a time through LDS.
    constexpr int kLanesPerRow = 64 / RW;
    const int i = lane / kLanesPerRow;
    const int prt = lane % kLanesPerRow;
    const uint32_t r = row0 + (uint32_t)i;
#pragma unroll
    for (int b = 0; b < NQ; ++b) {
        __syncthreads();
#pragma unroll
        for (int t = 0; t < RW; ++t) s_red[wave][t][lane] = acc[t][b];
        __syncthreads();
        acc_t v = 0;
#pragma unroll
        for (int t = 0; t < RW; ++t) v += s_red[wave][i][prt * RW + t];
#pragma unroll
        for (int off = 1; off < kLanesPerRow; off <<= 1) v += __shfl_xor(v, off);
        if (prt == 0 && r < R && (uint32_t)b < B)
            static_cast<acc_t*>(part)[((uint64_t)blockIdx.y * B + b) * R + r] = v;
    }
}

// Sum of the column splits; the field form reduces mod p.  Output element
// (r, b) goes to out[r * o_ldr + b * o_ldb].
template <bool EXACT>
__global__ void k_few_finish(const void* __restrict__ part, uint32_t R, uint32_t B, uint32_t S,
                             uint32_t p, uint32_t* __restrict__ out, uint64_t o_ldr,
                             uint64_t o_ldb) {
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (uint64_t)R * B) return;
    const uint32_t b = (uint32_t)(idx / R), r = (uint32_t)(idx % R);
    uint32_t* dst = out + (uint64_t)r * o_ldr + (uint64_t)b * o_ldb;
    if (EXACT) {
        uint64_t v = 0;
        for (uint32_t s = 0; s < S; ++s)
            v += static_cast<const uint64_t*>(part)[((uint64_t)s * B + b) * R + r];
        *dst = (uint32_t)(v % p);
    } else {
        uint32_t v = 0;
        for (uint32_t s = 0; s < S; ++s)
            v += static_cast<const uint32_t*>(part)[((uint64_t)s * B + b) * R + r];
        *dst = v;
    }
}

template <int NQ>
constexpr int few_rw() { return NQ == 4 ? 8 : 16; }

uint32_t few_nq(uint32_t B) { return B <= 1 ? 1u : (B <= 2 ? 2u : 4u); }

// Column splits for the few-query stream (as for k_answer1), and the
// partial buffer: splits x B x R accumulators (8 bytes, enough for both
// forms).
SplitPlan few_plan(const pir_db_t* db, uint32_t B) {
    const uint32_t rw = few_nq(B) == 4 ? 8u : 16u;
    return plan_splits(db, rw * kWaves);
}

template <int NQ, bool EXACT>
pir_status launch_few_t(const pir_db_t* db, const BatchIO& io, uint32_t B, uint32_t modulus,
                        void* ws, hipStream_t s) {
    constexpr int RW = few_rw<NQ>();
    constexpr uint32_t kRows = RW * kWaves;
    const SplitPlan pl = plan_splits(db, kRows);
    const uint32_t R = (uint32_t)db->rows, C = (uint32_t)db->cols;
    dim3 grid((R + kRows - 1) / kRows, pl.splits);
    if (db->aligned)
        k_answer_few<NQ, RW, true, EXACT><<<grid, kThreads, 0, s>>>(
            db->D, db->pitch, R, C, io.Q, io.q_ldj, io.q_ldb, B, pl.cols_per_split, ws);
    else
        k_answer_few<NQ, RW, false, EXACT><<<grid, kThreads, 0, s>>>(
            db->D, db->pitch, R, C, io.Q, io.q_ldj, io.q_ldb, B, pl.cols_per_split, ws);
    PIR_LAUNCH_CHECK();
    const uint64_t n = (uint64_t)R * B;
    k_few_finish<EXACT><<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(
        ws, R, B, pl.splits, modulus, io.out, io.o_ldr, io.o_ldb);
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

}  // namespace

size_t few_workspace_bytes(const pir_db_t* db, uint32_t B) {
    if (B == 0 || B > kFewMax) return 0;
    const SplitPlan pl = few_plan(db, B);
    return round_up((size_t)pl.splits * B * db->rows * 8, kWsAlign);
}

pir_status few_answer_batch(const pir_db_t* db, const BatchIO& io, uint32_t B, uint32_t modulus,
                            void* ws, size_t ws_bytes, hipStream_t s) {
    if (B == 0) return PIR_OK;
    if (B > kFewMax) return PIR_ERR_SHAPE;
    if (!ws || ws_bytes < few_workspace_bytes(db, B) || ((uintptr_t)ws % kWsAlign))
        return PIR_ERR_WORKSPACE;
    const bool exact = modulus != 0;
    switch (few_nq(B)) {
        case 1: return exact ? launch_few_t<1, true>(db, io, B, modulus, ws, s)
                             : launch_few_t<1, false>(db, io, B, modulus, ws, s);
        case 2: return exact ? launch_few_t<2, true>(db, io, B, modulus, ws, s)
                             : launch_few_t<2, false>(db, io, B, modulus, ws, s);
        default: return exact ? launch_few_t<4, true>(db, io, B, modulus, ws, s)
                              : launch_few_t<4, false>(db, io, B, modulus, ws, s);
    }
}

uint32_t gemv_variant_count() { return kNumGemv; }

const char* gemv_variant_name(uint32_t v) { return v < kNumGemv ? kGemv[v].name : nullptr; }

// Enough for every variant, so a workspace sized once serves any tuning.
size_t gemv_workspace_bytes(const pir_db_t* db) {
    size_t m = 0;
    for (uint32_t v = 0; v < kNumGemv; ++v) {
        const size_t b = split_bytes(db, kGemv[v].rows_per_wave * kWaves);
        m = b > m ? b : m;
    }
    return m;
}

pir_status gemv_answer(const pir_db_t* db, const uint32_t* q, uint32_t* a, void* ws,
                       size_t ws_bytes, hipStream_t s) {
    uint32_t v = db->variant[0];
    if (v >= kNumGemv) v = 0;
    return kGemv[v].launch(db, q, a, ws, ws_bytes, s);
}
