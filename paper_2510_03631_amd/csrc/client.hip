// Client side of LWE PIR on the GPU: query construction and decoding.
//
// Definition 1's client algorithms, in single-server LWE form:
//   query   q_b = A s_b + e_b + Delta u_{col_b}         (mod 2^32)
//   decode  m_b[r] = ((a_b[r] - (H s_b)[r] + Delta/2) mod 2^32) >> 24
// with Delta = 2^32 / 256.  Both are products of a word matrix (A: C x n, or
// H: R x n) with a batch of secrets over Z/2^32, one row dot product per
// output, followed by an elementwise epilogue.
//
// k_rowdot: one wave per 4 matrix rows for batches of secrets (1 for a few
// secrets or on the word path), so every secret word loaded serves 4 rows.
// Per 1024-word chunk a lane holds 16
// words of the row, 4 x 16 bytes at 4 * lane + 256 e (VEC: n % 4 == 0 and
// aligned rows) or single words at lane + 64 e, so every load instruction
// is coalesced, and multiplies them with the same words of up to 16 secrets
// at a time (v_mul_lo_u32 / add, natural 2^32 wrap); the 16 per-lane partial
// sums are transposed through LDS and finished with lane shuffles, so lane
// (b, part) ends with output (b, row).
#include <string.h>

#include <new>

#include "qpir_internal.h"

namespace {

constexpr int kCWaves = 4;
constexpr int kBChunk = 16;     // secrets per pass over a row
constexpr uint32_t kDelta = 1u << 24;
constexpr uint32_t kHalfDelta = 1u << 23;

enum Epilogue { kQuery = 0, kDecode = 1 };

// The 16 words a lane covers in a 1024-word chunk starting at k0.
template <bool VEC>
__device__ inline void load16(const uint32_t* __restrict__ row, uint32_t k0, uint32_t n, int lane,
                              uint32_t (&w)[16]) {
    if constexpr (VEC) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t k = k0 + 256u * e + 4u * lane;
            const u32x4 v = k < n ? *reinterpret_cast<const u32x4*>(row + k) : u32x4{0u, 0u, 0u, 0u};
            w[4 * e + 0] = v.x;
            w[4 * e + 1] = v.y;
            w[4 * e + 2] = v.z;
            w[4 * e + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const uint32_t k = k0 + 64u * e + lane;
            w[e] = k < n ? row[k] : 0u;
        }
    }
}

// y[b][r] = sum_k M[r][k] * X[b][k]; then the epilogue.  A wave takes RB
// consecutive rows at once, so each secret word it loads serves RB rows.
template <int EPI, bool VEC, int RB>
__global__ __launch_bounds__(64 * kCWaves) void k_rowdot(
    const uint32_t* __restrict__ M, uint32_t rows, uint32_t n,
    const uint32_t* __restrict__ X, uint32_t B,
    const int32_t* __restrict__ E, const uint32_t* __restrict__ cols,   // query
    const uint32_t* __restrict__ ans,                                    // decode
    uint32_t* __restrict__ out_words, uint8_t* __restrict__ out_bytes) {
    __shared__ uint32_t s_red[kCWaves][kBChunk][65];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t nwaves = gridDim.x * kCWaves;
    for (uint32_t r0 = (blockIdx.x * kCWaves + wave) * RB; r0 < rows; r0 += nwaves * RB) {
        // Rows past the end re-read the last row; their sums are dropped.
        const uint32_t* mrow[RB];
#pragma unroll
        for (int i = 0; i < RB; ++i) mrow[i] = M + (uint64_t)min(r0 + i, rows - 1) * n;
        for (uint32_t b0 = 0; b0 < B; b0 += kBChunk) {
            uint32_t acc[RB][kBChunk];
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int b = 0; b < kBChunk; ++b) acc[i][b] = 0;
            for (uint32_t k0 = 0; k0 < n; k0 += 1024) {
                uint32_t m[RB][16];
#pragma unroll
                for (int i = 0; i < RB; ++i) load16<VEC>(mrow[i], k0, n, lane, m[i]);
#pragma unroll
                for (int b = 0; b < kBChunk; ++b) {
                    if (b0 + b < B) {
                        uint32_t x[16];
                        load16<VEC>(X + (uint64_t)(b0 + b) * n, k0, n, lane, x);
#pragma unroll
                        for (int i = 0; i < RB; ++i) {
                            uint32_t a = acc[i][b];
#pragma unroll
                            for (int e = 0; e < 16; ++e) a += m[i][e] * x[e];
                            acc[i][b] = a;
                        }
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                const uint32_t r = r0 + i;
                if (r >= rows) break;   // uniform over the wave
                // Row sums: lane (b = lane / 4, part = lane % 4) adds 16 partials.
#pragma unroll
                for (int b = 0; b < kBChunk; ++b) s_red[wave][b][lane] = acc[i][b];
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const int b = lane >> 2, part = lane & 3;
                uint32_t v = 0;
#pragma unroll
                for (int t = 0; t < 16; ++t) v += s_red[wave][b][part * 16 + t];
                v += __shfl_xor(v, 1);
                v += __shfl_xor(v, 2);
                __builtin_amdgcn_wave_barrier();
                const uint32_t bb = b0 + (uint32_t)b;
                if (part == 0 && bb < B) {
                    if (EPI == kQuery) {
                        uint32_t q = v + (uint32_t)E[(uint64_t)bb * rows + r];
                        if (r == cols[bb]) q += kDelta;
                        out_words[(uint64_t)bb * rows + r] = q;
                    } else {
                        const uint32_t d = ans[(uint64_t)bb * rows + r] - v + kHalfDelta;
                        out_bytes[(uint64_t)bb * rows + r] = (uint8_t)(d >> 24);
                    }
                }
            }
        }
    }
}

// 16-byte loads need n % 4 == 0 and 16-byte aligned matrix and secrets.
bool vec_ok(const void* M, const void* X, uint32_t n) {
    return n % 4 == 0 && (uintptr_t)M % 16 == 0 && (uintptr_t)X % 16 == 0;
}

// Rows per wave: 4 on the 16-byte path for more than kFewSecrets secrets
// (each secret word then serves 4 rows), else 1.  Few secrets leave the
// kernel bound by reading the matrix, where more waves in flight count
// more (32768 x 1024, one secret: 24.9 us with one row per wave, 29.5 us
// with four; 64 secrets: 286 us and 205 us).
constexpr int kRowsVec = 4;
constexpr uint32_t kFewSecrets = 4;

uint32_t grid_for(uint32_t rows, int rb) {
    const uint64_t per = (uint64_t)kCWaves * rb;
    const uint64_t blocks = (rows + per - 1) / per;
    return blocks < 16384 ? (uint32_t)blocks : 16384u;
}

// ---------------------------------------------------------------- matrix-core path
// Over Z/2^32 a word matrix is the sum of its byte planes, M = sum_i 2^(8i)
// M_i, so M x = [M_0 | M_1 | M_2 | M_3] [x; 2^8 x; 2^16 x; 2^24 x]: a byte
// matrix of 4n columns times a word vector of 4n entries, which is exactly
// the Answer product D q.  A prepared client matrix holds the byte planes
// (rows x 4n bytes, the same size as M) under a database handle, and a batch
// of secrets runs on the matrix-core batched Answer, followed by the query
// or decode epilogue.

constexpr uint32_t kClientMatMagic = 0x434D4154u;   // "CMAT"

// planes[r][i n + k] = byte i of M[r][k]; one thread per word.
__global__ void k_byte_planes(const uint32_t* __restrict__ M, uint64_t words, uint32_t n,
                              uint8_t* __restrict__ planes) {
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= words) return;
    const uint64_t r = idx / n, k = idx % n;
    const uint32_t w = M[idx];
    uint8_t* row = planes + r * 4u * n;
#pragma unroll
    for (int i = 0; i < 4; ++i) row[(uint64_t)i * n + k] = (uint8_t)(w >> (8 * i));
}

// The batched Answer's operand for the secrets against the planes,
// xs_b = [x_b; 2^8 x_b; 2^16 x_b; 2^24 x_b] (mod 2^32, 4n words), written
// straight in its wide limb layout: block b writes the four limb rows of
// query b over all Cp columns (zero past 4n, all zero for the padding
// queries b >= B) and the exact sum of xs_b, so no clearing pass and no
// atomics are needed.
__global__ __launch_bounds__(256) void k_client_planes(const uint32_t* __restrict__ X,
                                                       uint32_t B, uint32_t n, uint32_t Cp,
                                                       int8_t* __restrict__ QL,
                                                       uint64_t* __restrict__ colsum) {
    __shared__ uint64_t s_sum[256];
    const uint32_t b = blockIdx.x;
    const bool live = b < B;
    const uint32_t K = 4u * n;
    const uint32_t nrow = (b / 32u) * 128u + b % 32u;   // limb 0 row; limb L adds 32 L
    uint64_t sum = 0;
    for (uint32_t k = 4u * threadIdx.x; k < Cp; k += 4u * blockDim.x) {
        uint32_t word[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t j = k + (uint32_t)c;
            uint32_t w = 0;
            if (live && j < K) {
                w = X[(uint64_t)b * n + j % n] << (8u * (j / n));
                sum += w;
            }
#pragma unroll
            for (int L = 0; L < 4; ++L) {
                const uint32_t byte = (live && j < K) ? (((w >> (8 * L)) & 0xFFu) ^ 0x80u) : 0u;
                word[L] |= byte << (8 * c);
            }
        }
#pragma unroll
        for (int L = 0; L < 4; ++L)
            *reinterpret_cast<uint32_t*>(QL + ql_row(nrow + 32u * L, Cp) + ql_col(k)) = word[L];
    }
    s_sum[threadIdx.x] = sum;
    __syncthreads();
    for (uint32_t h = blockDim.x / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) s_sum[threadIdx.x] += s_sum[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) colsum[b] = live ? s_sum[0] : 0u;
}

// Query epilogue, in place on the product: Qt[b][j] += E[b][j] (+ Delta at
// the queried column).
__global__ void k_query_epilogue(uint32_t* __restrict__ Qt, uint32_t C, uint32_t B,
                                 const int32_t* __restrict__ E, const uint32_t* __restrict__ cols) {
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (uint64_t)B * C) return;
    const uint32_t b = (uint32_t)(idx / C), j = (uint32_t)(idx % C);
    uint32_t q = Qt[idx] + (uint32_t)E[idx];
    if (j == cols[b]) q += kDelta;
    Qt[idx] = q;
}

// Decode epilogue: out[b][r] = ((ans[b][r] - Y[b][r] + Delta/2) mod 2^32) >> 24.
__global__ void k_decode_epilogue(const uint32_t* __restrict__ Y, const uint32_t* __restrict__ ans,
                                  uint64_t count, uint8_t* __restrict__ out) {
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= count) return;
    out[idx] = (uint8_t)((ans[idx] - Y[idx] + kHalfDelta) >> 24);
}

// One thread per element in 256-thread blocks: at most 2^31 - 1 blocks.
constexpr uint64_t kMaxGridWords = 0x7FFFFFFFull * 256u;
uint32_t grid1d(uint64_t n) { return (uint32_t)((n + 255) / 256); }

}  // namespace

struct pir_client_mat {
    uint32_t magic;
    uint32_t rows, n;
    int device;
    uint8_t* planes;   // rows x 4n bytes, owned
    pir_db_t* db;      // handle over the planes
};

namespace {

bool mat_ok(const pir_client_mat_t* m) { return m && m->magic == kClientMatMagic; }

// Workspace layout of a batch of B: the secrets' limb planes and column
// sums, the product (decode only), then the batched Answer's workspace.
struct MatWs {
    size_t planes_off, y_off, ans_off, total;
};

MatWs mat_ws(const pir_client_mat_t* m, uint32_t B, bool decode) {
    MatWs w;
    w.planes_off = 0;
    w.y_off = round_up(mfma_planes_bytes(m->db, B), kWsAlign);
    w.ans_off = w.y_off + (decode ? round_up((size_t)B * m->rows * 4u, kWsAlign) : 0);
    w.total = w.ans_off + pir_workspace_bytes(m->db, B);
    return w;
}

// Y[b] = M X[b] for the B secrets into y (B x rows words); `plan` made with
// pre-ingested planes.
pir_status mat_product(pir_client_mat_t* m, const uint32_t* X, uint32_t B, uint32_t* y,
                       uint8_t* ws, const MatWs& w, const BatchPlan& plan, hipStream_t st) {
    uint8_t* planes = ws + w.planes_off;
    k_client_planes<<<plan.Bp, 256, 0, st>>>(X, B, m->n, plan.Cp,
                                             reinterpret_cast<int8_t*>(planes),
                                             reinterpret_cast<uint64_t*>(planes + plan.colsum_off));
    PIR_LAUNCH_CHECK();
    const BatchIO io{nullptr, 1, 4u * m->n, y, 1, m->rows};   // query-major answers
    return mfma_run_batch(m->db, io, B, nullptr, 0, plan, ws + w.ans_off, planes, st);
}

}  // namespace

extern "C" {

pir_status pir_client_mat_open(const uint32_t* d_M, uint32_t rows, uint32_t n,
                               pir_stream_t stream, pir_client_mat_t** out) {
    if (!d_M || !out) return PIR_ERR_INVALID_ARG;
    if (rows == 0 || n == 0 || rows > kMaxDim || (uint64_t)4 * n > kMaxDim ||
        (uint64_t)rows * n > kMaxGridWords)
        return PIR_ERR_SHAPE;
    if (!current_is_gfx950()) return PIR_ERR_UNSUPPORTED;
    pir_client_mat_t* m = new (std::nothrow) pir_client_mat_t();
    if (!m) return PIR_ERR_NO_MEMORY;
    m->rows = rows;
    m->n = n;
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        return PIR_ERR_DEVICE;
    }
    const uint64_t bytes = (uint64_t)rows * 4u * n;
    if (hipMalloc((void**)&m->planes, bytes) != hipSuccess) {
        delete m;
        return PIR_ERR_NO_MEMORY;
    }
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const uint64_t words = (uint64_t)rows * n;
    k_byte_planes<<<grid1d(words), 256, 0, st>>>(d_M, words, n, m->planes);
    pir_status s = hipGetLastError() == hipSuccess ? PIR_OK : PIR_ERR_DEVICE;
    if (s == PIR_OK) s = pir_db_open(m->planes, rows, 4u * n, 4u * n, stream, &m->db);
    if (s != PIR_OK) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(m->planes);
        delete m;
        return s;
    }
    // The product's default tile: a 128 x 128 ring with two 128-byte stages,
    // two workgroups per CU (the client product has K = 4n, small beside
    // its rows).  Measured at 32768 x 1024 words, whole query call: 16
    // secrets 39 us against 44 us with the database default, 64 secrets 54
    // against 60 us.  pir_client_mat_set_variant overrides it.
    for (uint32_t v = 1; v < mfma_variant_count(); ++v) {
        if (strcmp(mfma_variant_name(v), "ring_128x128_k128_s2") != 0) continue;
        for (uint32_t b = 8; b <= kMaxBatch; b *= 2) (void)pir_db_set_variant(m->db, b, v);
    }
    m->magic = kClientMatMagic;
    *out = m;
    return PIR_OK;
}

pir_status pir_client_mat_close(pir_client_mat_t* m) {
    if (!m) return PIR_OK;
    if (!mat_ok(m)) return PIR_ERR_INVALID_ARG;
    pir_status st = pir_db_close(m->db);   // synchronizes the device
    if (hipFree(m->planes) != hipSuccess) st = PIR_ERR_DEVICE;
    m->magic = 0;
    delete m;
    return st;
}

pir_status pir_client_mat_set_variant(pir_client_mat_t* m, uint32_t batch, uint32_t variant) {
    if (!mat_ok(m) || batch == 0 || (batch & PIR_VARIANT_ROWS)) return PIR_ERR_INVALID_ARG;
    return pir_db_set_variant(m->db, batch, variant);
}

size_t pir_client_mat_workspace_bytes(const pir_client_mat_t* m, uint32_t B) {
    if (!mat_ok(m) || B == 0 || B > kMaxBatch) return 0;
    return mat_ws(m, B, true).total;
}

pir_status pir_client_query_mat(pir_client_mat_t* A, const uint32_t* d_S, const int32_t* d_E,
                                const uint32_t* d_cols, uint32_t B, uint32_t* d_Qt, void* d_ws,
                                size_t ws_bytes, pir_stream_t stream) {
    if (!mat_ok(A) || !d_S || !d_E || !d_cols || !d_Qt) return PIR_ERR_INVALID_ARG;
    if (B == 0 || B > kMaxBatch || (uint64_t)B * A->rows > kMaxGridWords ||
        (uint64_t)B * A->n > kMaxGridWords)
        return PIR_ERR_SHAPE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != A->device) return PIR_ERR_INVALID_ARG;
    if (!d_ws || ws_bytes < pir_client_mat_workspace_bytes(A, B) || (uintptr_t)d_ws % kWsAlign)
        return PIR_ERR_WORKSPACE;
    const MatWs w = mat_ws(A, B, false);
    const hipStream_t st = static_cast<hipStream_t>(stream);
    BatchPlan plan;   // every check of the product before anything is enqueued
    pir_status s = mfma_plan_batch(A->db, B, nullptr, 0, 0, true, &plan);
    if (s != PIR_OK) return s;
    s = mat_product(A, d_S, B, d_Qt, static_cast<uint8_t*>(d_ws), w, plan, st);
    if (s != PIR_OK) return s;
    k_query_epilogue<<<grid1d((uint64_t)B * A->rows), 256, 0, st>>>(d_Qt, A->rows, B, d_E, d_cols);
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

pir_status pir_client_decode_mat(pir_client_mat_t* H, const uint32_t* d_S,
                                 const uint32_t* d_answers, uint32_t B, uint8_t* d_out,
                                 void* d_ws, size_t ws_bytes, pir_stream_t stream) {
    if (!mat_ok(H) || !d_S || !d_answers || !d_out) return PIR_ERR_INVALID_ARG;
    if (B == 0 || B > kMaxBatch || (uint64_t)B * H->rows > kMaxGridWords ||
        (uint64_t)B * H->n > kMaxGridWords)
        return PIR_ERR_SHAPE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != H->device) return PIR_ERR_INVALID_ARG;
    if (!d_ws || ws_bytes < pir_client_mat_workspace_bytes(H, B) || (uintptr_t)d_ws % kWsAlign)
        return PIR_ERR_WORKSPACE;
    const MatWs w = mat_ws(H, B, true);
    const hipStream_t st = static_cast<hipStream_t>(stream);
    BatchPlan plan;
    pir_status s = mfma_plan_batch(H->db, B, nullptr, 0, 0, true, &plan);
    if (s != PIR_OK) return s;
    uint8_t* ws = static_cast<uint8_t*>(d_ws);
    uint32_t* y = reinterpret_cast<uint32_t*>(ws + w.y_off);
    s = mat_product(H, d_S, B, y, ws, w, plan, st);
    if (s != PIR_OK) return s;
    const uint64_t count = (uint64_t)B * H->rows;
    k_decode_epilogue<<<grid1d(count), 256, 0, st>>>(y, d_answers, count, d_out);
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

pir_status pir_client_query(const uint32_t* d_A, uint32_t C, uint32_t n, const uint32_t* d_S,
                            const int32_t* d_E, const uint32_t* d_cols, uint32_t B,
                            uint32_t* d_Qt, pir_stream_t stream) {
    if (!d_A || !d_S || !d_E || !d_cols || !d_Qt) return PIR_ERR_INVALID_ARG;
    if (C == 0 || n == 0 || B == 0 || C > kMaxDim || n > kMaxDim || B > kMaxBatch)
        return PIR_ERR_SHAPE;
    if (!current_is_gfx950()) return PIR_ERR_UNSUPPORTED;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (vec_ok(d_A, d_S, n) && B > kFewSecrets)
        k_rowdot<kQuery, true, kRowsVec><<<grid_for(C, kRowsVec), 64 * kCWaves, 0, st>>>(
            d_A, C, n, d_S, B, d_E, d_cols, nullptr, d_Qt, nullptr);
    else if (vec_ok(d_A, d_S, n))
        k_rowdot<kQuery, true, 1><<<grid_for(C, 1), 64 * kCWaves, 0, st>>>(
            d_A, C, n, d_S, B, d_E, d_cols, nullptr, d_Qt, nullptr);
    else
        k_rowdot<kQuery, false, 1><<<grid_for(C, 1), 64 * kCWaves, 0, st>>>(
            d_A, C, n, d_S, B, d_E, d_cols, nullptr, d_Qt, nullptr);
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

pir_status pir_client_decode(const uint32_t* d_H, uint32_t R, uint32_t n, const uint32_t* d_S,
                             const uint32_t* d_answers, uint32_t B, uint8_t* d_out,
                             pir_stream_t stream) {
    if (!d_H || !d_S || !d_answers || !d_out) return PIR_ERR_INVALID_ARG;
    if (R == 0 || n == 0 || B == 0 || R > kMaxDim || n > kMaxDim || B > kMaxBatch)
        return PIR_ERR_SHAPE;
    if (!current_is_gfx950()) return PIR_ERR_UNSUPPORTED;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (vec_ok(d_H, d_S, n) && B > kFewSecrets)
        k_rowdot<kDecode, true, kRowsVec><<<grid_for(R, kRowsVec), 64 * kCWaves, 0, st>>>(
            d_H, R, n, d_S, B, nullptr, nullptr, d_answers, nullptr, d_out);
    else if (vec_ok(d_H, d_S, n))
        k_rowdot<kDecode, true, 1><<<grid_for(R, 1), 64 * kCWaves, 0, st>>>(
            d_H, R, n, d_S, B, nullptr, nullptr, d_answers, nullptr, d_out);
    else
        k_rowdot<kDecode, false, 1><<<grid_for(R, 1), 64 * kCWaves, 0, st>>>(
            d_H, R, n, d_S, B, nullptr, nullptr, d_answers, nullptr, d_out);
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

}  // extern "C"
