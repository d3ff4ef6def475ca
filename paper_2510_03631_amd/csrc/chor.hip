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
// * per 32-row block the group's 32 query bits per query are loaded once
//   (wave-uniform); a row that no query of the group selects is never read;
//   the selected rows of 8 consecutive rows are loaded back to back (up to
//   8 KiB per wave in flight), then XORed into the accumulators of the
//   queries that select them, with wave-uniform branches (only selected
//   (row, query) pairs cost VALU work);
// * workgroups are numbered slab-major and dealt to XCDs in contiguous
//   ranges, so the query groups of one slab share its rows in L2;
// * slabs combine into the output with atomicXor (XOR is associative and
//   commutative, so the result does not depend on the order); the output is
//   cleared first by a fill kernel.
#include <string.h>

#include "qpir_internal.h"

namespace {

constexpr int kG = 16;            // queries per workgroup
constexpr int kThreads = 256;
constexpr uint32_t kChunkWords = 4 * kThreads;

__global__ void k_chor_zero(uint32_t* __restrict__ p, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

template <bool VEC>
__device__ inline u32x4 load_words(const uint32_t* row, uint32_t w, uint32_t W) {
    if (VEC) return *reinterpret_cast<const u32x4*>(row + w);   // W % 4 == 0, aligned
    return u32x4{w < W ? row[w] : 0u, w + 1 < W ? row[w + 1] : 0u,
                 w + 2 < W ? row[w + 2] : 0u, w + 3 < W ? row[w + 3] : 0u};
}

template <bool VEC>
__global__ __launch_bounds__(kThreads) void k_chor(const uint32_t* __restrict__ DB, uint64_t pitch,
                                                   uint32_t rows, uint32_t W,
                                                   const uint32_t* __restrict__ Q, uint32_t qwords,
                                                   uint32_t B, uint32_t slab_rows,
                                                   uint32_t n_groups, uint32_t* __restrict__ out) {
    uint32_t bid = blockIdx.x;
    {
        const uint32_t per = gridDim.x / 8u;
        if (bid < per * 8u) bid = (bid % 8u) * per + bid / 8u;
    }
    const uint32_t slab = bid / n_groups;
    const uint32_t grp = bid % n_groups;
    const uint32_t r0 = slab * slab_rows;
    const uint32_t r1 = min(rows, r0 + slab_rows);
    const uint32_t b0 = grp * kG;
    const uint32_t nb = min((uint32_t)kG, B - b0);

    for (uint32_t c0 = 0; c0 < W; c0 += kChunkWords) {
        const uint32_t w = c0 + 4u * threadIdx.x;
        const bool active = w < W;
        u32x4 acc[kG];
#pragma unroll
        for (int g = 0; g < kG; ++g) acc[g] = u32x4{0, 0, 0, 0};

        for (uint32_t r = r0; r < r1; r += 32) {
            // This block's selector bits for each query of the group.
            uint32_t qb[kG];
            uint32_t any = 0;
            const uint32_t valid = (r1 - r >= 32) ? 0xFFFFFFFFu : ((1u << (r1 - r)) - 1u);
#pragma unroll
            for (int g = 0; g < kG; ++g) {
                qb[g] = (uint32_t)g < nb
                            ? __builtin_amdgcn_readfirstlane(Q[(uint64_t)(b0 + g) * qwords + r / 32]) & valid
                            : 0u;
                any |= qb[g];
            }
            if (!any) continue;
#pragma unroll
            for (int j0 = 0; j0 < 32; j0 += 8) {
                if (!((any >> j0) & 0xFFu)) continue;
                u32x4 d[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    d[k] = u32x4{0, 0, 0, 0};
                    if (((any >> (j0 + k)) & 1u) && active)
                        d[k] = load_words<VEC>(DB + (uint64_t)(r + j0 + k) * pitch, w, W);
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
#pragma unroll
                    for (int g = 0; g < kG; ++g)
                        if ((qb[g] >> (j0 + k)) & 1u) acc[g] ^= d[k];
                }
            }
        }
        if (active) {
#pragma unroll
            for (int g = 0; g < kG; ++g) {
                if ((uint32_t)g >= nb) break;
                uint32_t* o = out + (uint64_t)(b0 + g) * W + w;
                const uint32_t v[4] = {acc[g].x, acc[g].y, acc[g].z, acc[g].w};
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (w + e < W && v[e]) atomicXor(o + e, v[e]);
            }
        }
    }
}

bool current_is_gfx950() {
    int dev = -1;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return false;
    return strncmp(prop.gcnArchName, "gfx950", 6) == 0;
}

}  // namespace

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
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint64_t n_out = (uint64_t)B * words;
    k_chor_zero<<<(uint32_t)((n_out + 255) / 256), 256, 0, s>>>(d_out, n_out);
    PIR_LAUNCH_CHECK();
    const uint32_t qwords = (rows + 31) / 32;
    const uint32_t n_groups = (B + kG - 1) / kG;
    // About 2048 workgroups: slabs of a multiple of 32 rows.
    uint64_t slab = ((uint64_t)rows * n_groups + 2047) / 2048;
    slab = (slab + 31) / 32 * 32;
    if (slab < 32) slab = 32;
    const uint64_t n_slabs = (rows + slab - 1) / slab;
    const uint64_t blocks = n_slabs * n_groups;
    if (blocks > 0x7FFFFFFFull) return PIR_ERR_SHAPE;
    const bool vec = ((uintptr_t)d_DB % 16 == 0) && (words % 4 == 0) && (row_pitch_words % 4 == 0);
    if (vec)
        k_chor<true><<<(uint32_t)blocks, kThreads, 0, s>>>(d_DB, row_pitch_words, rows, words, d_Q,
                                                           qwords, B, (uint32_t)slab, n_groups,
                                                           d_out);
    else
        k_chor<false><<<(uint32_t)blocks, kThreads, 0, s>>>(d_DB, row_pitch_words, rows, words, d_Q,
                                                            qwords, B, (uint32_t)slab, n_groups,
                                                            d_out);
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

}  // extern "C"
