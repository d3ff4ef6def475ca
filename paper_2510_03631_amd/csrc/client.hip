// Client side of LWE PIR on the GPU: query construction and decoding.
//
// Definition 1's client algorithms, in single-server LWE form:
//   query   q_b = A s_b + e_b + Delta u_{col_b}         (mod 2^32)
//   decode  m_b[r] = ((a_b[r] - (H s_b)[r] + Delta/2) mod 2^32) >> 24
// with Delta = 2^32 / 256.  Both are products of a word matrix (A: C x n, or
// H: R x n) with a batch of secrets over Z/2^32, one row dot product per
// output, followed by an elementwise epilogue.
//
// k_rowdot: one wave per matrix row.  Per 1024-word chunk a lane holds the
// words lane, lane + 64, ... (every load instruction coalesced) and
// multiplies them with the same words of up to 16 secrets at a time
// (v_mul_lo_u32 / add, natural 2^32 wrap); the 16 per-lane partial sums are
// transposed through LDS and finished with lane shuffles, so lane (b, part)
// ends with output (b, row).
#include <string.h>

#include "qpir_internal.h"

namespace {

constexpr int kCWaves = 4;
constexpr int kBChunk = 16;     // secrets per pass over a row
constexpr uint32_t kDelta = 1u << 24;
constexpr uint32_t kHalfDelta = 1u << 23;

enum Epilogue { kQuery = 0, kDecode = 1 };

// y[b][r] = sum_k M[r][k] * X[b][k]; then the epilogue.
template <int EPI>
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
    for (uint32_t r = blockIdx.x * kCWaves + wave; r < rows; r += nwaves) {
        const uint32_t* mrow = M + (uint64_t)r * n;
        for (uint32_t b0 = 0; b0 < B; b0 += kBChunk) {
            uint32_t acc[kBChunk];
#pragma unroll
            for (int b = 0; b < kBChunk; ++b) acc[b] = 0;
            for (uint32_t k0 = 0; k0 < n; k0 += 1024) {
                uint32_t m[16];
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const uint32_t k = k0 + 64u * e + lane;
                    m[e] = k < n ? mrow[k] : 0u;
                }
#pragma unroll
                for (int b = 0; b < kBChunk; ++b) {
                    if (b0 + b < B) {
                        const uint32_t* x = X + (uint64_t)(b0 + b) * n;
                        uint32_t a = acc[b];
#pragma unroll
                        for (int e = 0; e < 16; ++e) {
                            const uint32_t k = k0 + 64u * e + lane;
                            a += m[e] * (k < n ? x[k] : 0u);
                        }
                        acc[b] = a;
                    }
                }
            }
            // Row sums: lane (b = lane / 4, part = lane % 4) adds 16 partials.
#pragma unroll
            for (int b = 0; b < kBChunk; ++b) s_red[wave][b][lane] = acc[b];
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

uint32_t grid_for(uint32_t rows) {
    const uint32_t blocks = (rows + kCWaves - 1) / kCWaves;
    return blocks < 16384 ? blocks : 16384;
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
    k_rowdot<kQuery><<<grid_for(C), 64 * kCWaves, 0, static_cast<hipStream_t>(stream)>>>(
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
    k_rowdot<kDecode><<<grid_for(R), 64 * kCWaves, 0, static_cast<hipStream_t>(stream)>>>(
        d_H, R, n, d_S, B, nullptr, nullptr, d_answers, nullptr, d_out);
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

}  // extern "C"
