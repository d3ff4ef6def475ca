// CIP-PIR, the OOP instantiation (Section 5.1, full instantiation; proof of
// Lemma 2): offline seed/value pairs and the online flip-chunk response.
//
// A server's local database is t chunks of k blocks (its flip chunk first,
// then t - 1 non-flip chunks), each block W 32-bit words, rows `pitch` words
// apart.
// * Offline, for each of `count` seeds: A = XOR of the non-flip blocks
//   (local rows k .. t k - 1) selected by the seed's PRG expansion, k(t-1)
//   bits.
// * Online, for each of B queries: out = A xor XOR of the flip-chunk blocks
//   (local rows 0 .. k - 1) its k-bit sub-query selects.
// Both are the XOR kernel of Chor PIR over a row range; the online call
// starts its accumulation from A instead of zero.
//
// PRG: ChaCha20 (RFC 8439 block function).  The 8-word seed is the key, the
// nonce is zero and the block counter counts 64-byte blocks from 0; keystream
// word w is selector word w (bit j selects non-flip block 32 w + j).  The
// paper asks for a secure PRG; ChaCha20 is this library's choice.
#include "qpir_internal.h"

namespace {

__device__ inline uint32_t rotl(uint32_t x, int n) { return (x << n) | (x >> (32 - n)); }

__device__ inline void quarter(uint32_t& a, uint32_t& b, uint32_t& c, uint32_t& d) {
    a += b; d = rotl(d ^ a, 16);
    c += d; b = rotl(b ^ c, 12);
    a += b; d = rotl(d ^ a, 8);
    c += d; b = rotl(b ^ c, 7);
}

// One thread per (seed e, 64-byte keystream block j): words 16 j .. 16 j + 15
// of seed e's output, nwords per seed; the last word keeps only the bits of
// `tail_mask`.
__global__ __launch_bounds__(256) void k_chacha(const uint32_t* __restrict__ seeds, uint32_t count,
                                                uint32_t nwords, uint32_t tail_mask,
                                                uint32_t* __restrict__ out) {
    const uint32_t nblk = (nwords + 15) / 16;
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (uint64_t)count * nblk) return;
    const uint32_t e = (uint32_t)(gid / nblk), j = (uint32_t)(gid % nblk);
    uint32_t in[16];
    in[0] = 0x61707865u; in[1] = 0x3320646eu; in[2] = 0x79622d32u; in[3] = 0x6b206574u;
#pragma unroll
    for (int w = 0; w < 8; ++w) in[4 + w] = seeds[(uint64_t)e * 8 + w];
    in[12] = j;
    in[13] = 0; in[14] = 0; in[15] = 0;
    uint32_t x[16];
#pragma unroll
    for (int w = 0; w < 16; ++w) x[w] = in[w];
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        quarter(x[0], x[4], x[8], x[12]);
        quarter(x[1], x[5], x[9], x[13]);
        quarter(x[2], x[6], x[10], x[14]);
        quarter(x[3], x[7], x[11], x[15]);
        quarter(x[0], x[5], x[10], x[15]);
        quarter(x[1], x[6], x[11], x[12]);
        quarter(x[2], x[7], x[8], x[13]);
        quarter(x[3], x[4], x[9], x[14]);
    }
    uint32_t* dst = out + (uint64_t)e * nwords;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
        const uint32_t idx = 16 * j + w;
        if (idx < nwords) {
            uint32_t v = x[w] + in[w];
            if (idx == nwords - 1) v &= tail_mask;
            dst[idx] = v;
        }
    }
}

pir_status launch_chacha(const uint32_t* d_seeds, uint32_t count, uint32_t bits, uint32_t* d_out,
                         hipStream_t s) {
    const uint32_t nwords = (bits + 31) / 32;
    const uint32_t tail = bits - 32 * (nwords - 1);
    const uint32_t tail_mask = tail == 32 ? 0xFFFFFFFFu : ((1u << tail) - 1u);
    const uint64_t threads = (uint64_t)count * ((nwords + 15) / 16);
    if ((threads + 255) / 256 > 0x7FFFFFFFull) return PIR_ERR_SHAPE;
    k_chacha<<<(uint32_t)((threads + 255) / 256), 256, 0, s>>>(d_seeds, count, nwords, tail_mask,
                                                               d_out);
    PIR_LAUNCH_CHECK();
    return PIR_OK;
}

bool oop_shape_ok(uint32_t k, uint32_t t, uint32_t words, uint64_t pitch) {
    return k >= 1 && t >= 1 && words >= 1 && pitch >= words && (uint64_t)k * t <= kMaxDim &&
           words <= kMaxDim;
}

}  // namespace

extern "C" {

pir_status pir_prg_expand(const uint32_t* d_seeds, uint32_t count, uint32_t bits, uint32_t* d_out,
                          pir_stream_t stream) {
    if (count == 0) return PIR_OK;
    if (!d_seeds || !d_out || bits == 0) return PIR_ERR_INVALID_ARG;
    if (count > kMaxBatch) return PIR_ERR_SHAPE;
    if (!current_is_gfx950()) return PIR_ERR_UNSUPPORTED;
    return launch_chacha(d_seeds, count, bits, d_out, static_cast<hipStream_t>(stream));
}

size_t pir_oop_workspace_bytes(uint32_t k, uint32_t t, uint32_t count) {
    if (t < 2 || k == 0) return 0;
    const uint64_t bits = (uint64_t)k * (t - 1);
    return round_up((size_t)count * ((bits + 31) / 32) * 4, kWsAlign);
}

pir_status pir_oop_offline(const uint32_t* d_DB, uint32_t k, uint32_t t, uint32_t words,
                           uint64_t row_pitch_words, const uint32_t* d_seeds, uint32_t count,
                           uint32_t* d_A, void* d_ws, size_t ws_bytes, pir_stream_t stream) {
    if (count == 0) return PIR_OK;
    if (!d_DB || !d_seeds || !d_A) return PIR_ERR_INVALID_ARG;
    if (!oop_shape_ok(k, t, words, row_pitch_words) || count > kMaxBatch) return PIR_ERR_SHAPE;
    const size_t need = pir_oop_workspace_bytes(k, t, count);
    if (need && (!d_ws || ws_bytes < need || (uintptr_t)d_ws % kWsAlign))
        return PIR_ERR_WORKSPACE;
    if (!current_is_gfx950()) return PIR_ERR_UNSUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (t == 1) return chor_init(d_A, nullptr, (uint64_t)count * words, s);   // no non-flip chunk
    const uint32_t rows = k * (t - 1);
    uint32_t* sel = static_cast<uint32_t*>(d_ws);
    pir_status st = launch_chacha(d_seeds, count, rows, sel, s);
    if (st != PIR_OK) return st;
    return chor_xor(d_DB + (uint64_t)k * row_pitch_words, rows, words, row_pitch_words, sel,
                    count, nullptr, d_A, s);
}

pir_status pir_oop_answer(const uint32_t* d_DB, uint32_t k, uint32_t words,
                          uint64_t row_pitch_words, const uint32_t* d_Q, uint32_t B,
                          const uint32_t* d_A, uint32_t* d_out, pir_stream_t stream) {
    if (B == 0) return PIR_OK;
    if (!d_DB || !d_Q || !d_A || !d_out) return PIR_ERR_INVALID_ARG;
    if (!oop_shape_ok(k, 1, words, row_pitch_words) || B > kMaxBatch) return PIR_ERR_SHAPE;
    if (!current_is_gfx950()) return PIR_ERR_UNSUPPORTED;
    return chor_xor(d_DB, k, words, row_pitch_words, d_Q, B, d_A, d_out,
                    static_cast<hipStream_t>(stream));
}

}  // extern "C"
