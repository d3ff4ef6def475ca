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

}  // namespace

extern "C" {

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
