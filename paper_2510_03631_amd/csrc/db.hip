// Database handle metadata and refresh kernels.
//
// The handle keeps one word per row, rowsum[r] = sum_j D[r][j] (exact for
// C < 2^24).  The matrix-core path works on centred bytes and limbs and adds
// back a term built from it (see answer_mfma.hip); it depends only on the
// database, so it is computed once when the handle is opened and again for
// the rows a refresh rewrites.
#include "qpir_internal.h"

namespace {

// One wave per row: byte sums through v_dot4_u32_u8 against 0x01010101.
template <bool VEC>
__global__ __launch_bounds__(256) void k_rowsum(const uint8_t* __restrict__ D, uint64_t pitch,
                                                 uint32_t R, uint32_t C,
                                                 const uint32_t* __restrict__ rows, uint32_t m,
                                                 uint32_t* __restrict__ rowsum) {
    const int lane = threadIdx.x & 63;
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    for (uint32_t i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < m; i += waves) {
        const uint32_t r = rows ? rows[i] : i;
        if (r >= R) continue;   // uniform across the wave
        const uint8_t* row = D + (uint64_t)r * pitch;
        uint32_t acc = 0;
        if (VEC) {
            uint32_t c = 16u * lane;
            for (; c + 16 <= C; c += 1024) {
                const u32x4 d = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(row + c));
                acc = __builtin_amdgcn_udot4(d.x, 0x01010101u, acc, false);
                acc = __builtin_amdgcn_udot4(d.y, 0x01010101u, acc, false);
                acc = __builtin_amdgcn_udot4(d.z, 0x01010101u, acc, false);
                acc = __builtin_amdgcn_udot4(d.w, 0x01010101u, acc, false);
            }
            for (; c < C; ++c) acc += row[c];   // this lane's ragged tail, at most 15 bytes
        } else {
            for (uint32_t c = lane; c < C; c += 64) acc += row[c];
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) rowsum[r] = acc;
    }
}

// Copy refreshed rows into place: block (i, y) copies part of new row i.
template <bool VEC>
__global__ __launch_bounds__(256) void k_scatter_rows(uint8_t* __restrict__ D, uint64_t pitch,
                                                      uint32_t R, uint32_t C,
                                                      const uint32_t* __restrict__ rows,
                                                      const uint8_t* __restrict__ src) {
    const uint32_t i = blockIdx.x;
    const uint32_t r = rows[i];
    if (r >= R) return;
    uint8_t* dst = D + (uint64_t)r * pitch;
    const uint8_t* s = src + (uint64_t)i * C;
    if (VEC) {
        const uint32_t c = (blockIdx.y * 256u + threadIdx.x) * 16u;
        if (c < C)   // C is a multiple of 16 on this path
            *reinterpret_cast<u32x4*>(dst + c) = *reinterpret_cast<const u32x4*>(s + c);
    } else {
        const uint32_t c0 = blockIdx.y * 4096u;
        for (uint32_t c = c0 + threadIdx.x; c < C && c < c0 + 4096u; c += 256) dst[c] = s[c];
    }
}

}  // namespace

pir_status launch_rowsum(const pir_db_t* db, const uint32_t* rows, uint32_t m, hipStream_t s) {
    if (m == 0) return PIR_OK;
    const uint32_t blocks = (uint32_t)((m + 3) / 4 < 8192 ? (m + 3) / 4 : 8192);
    if (db->aligned)
        k_rowsum<true><<<blocks, 256, 0, s>>>(db->D, db->pitch, (uint32_t)db->rows,
                                               (uint32_t)db->cols, rows, m, db->rowsum);
    else
        k_rowsum<false><<<blocks, 256, 0, s>>>(db->D, db->pitch, (uint32_t)db->rows,
                                                (uint32_t)db->cols, rows, m, db->rowsum);
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

pir_status launch_scatter_rows(const pir_db_t* db, const uint32_t* rows, uint32_t m,
                               const uint8_t* src, hipStream_t s) {
    if (m == 0) return PIR_OK;
    const uint32_t C = (uint32_t)db->cols;
    const bool vec = db->aligned && (C % 16 == 0) && ((uintptr_t)src % 16 == 0);
    if (vec) {
        dim3 grid(m, (C / 16 + 255) / 256);
        k_scatter_rows<true><<<grid, 256, 0, s>>>(db->D, db->pitch, (uint32_t)db->rows, C, rows,
                                                  src);
    } else {
        dim3 grid(m, (C + 4095) / 4096);
        k_scatter_rows<false><<<grid, 256, 0, s>>>(db->D, db->pitch, (uint32_t)db->rows, C, rows,
                                                   src);
    }
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}
