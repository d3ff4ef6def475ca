// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <algorithm>
#include <atomic>

#include "qpir.h"

constexpr int kBuckets = 24;   // batch-size buckets: 0 = single query, k = B in (2^(k-2), 2^(k-1)]

struct pir_db {
    uint32_t magic;        // kDbMagic while open
    uint8_t* D;            // borrowed database bytes
    uint64_t rows, cols, pitch;
    uint32_t* rowsum;      // device, rows words: sum_j D[r][j]
    int device;
    bool aligned;          // D and pitch are multiples of 16
    uint8_t variant[kBuckets];        // kernel variant per batch bucket (0 = built-in choice)
    uint8_t variant_rows[kBuckets];   // the same for row-gathered products
    // Cached split-K bound per padded-batch bucket: (N << 40) | (splits x rows),
    // 0 when not yet computed (see answer_mfma.hip).
    mutable std::atomic<uint64_t> split_rows[kBuckets];
};

constexpr uint32_t kDbMagic = 0x51504952u;   // "QPIR"
constexpr uint64_t kMaxDim = (1ull << 31) - 1;
constexpr size_t kWsAlign = 256;
constexpr uint32_t kMaxBatch = 1u << 20;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

inline bool db_ok(const pir_db_t* db) { return db && db->magic == kDbMagic; }

inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bucket of a batch size: 0 for the single-query entry point (batch == 0),
// otherwise 1 + ceil(log2(B)).
inline int batch_bucket(uint32_t batch) {
    if (batch == 0) return 0;
    int k = 0;
    while ((1u << k) < batch && k < 31) ++k;
    return k + 1 < kBuckets ? k + 1 : kBuckets - 1;
}

#define PIR_LAUNCH_CHECK()                                   \
    do {                                                     \
        if (hipGetLastError() != hipSuccess) return PIR_ERR_DEVICE; \
    } while (0)

// Query matrix and answer matrix of a batched call, as word strides:
// query b word j at Q[j * q_ldj + b * q_ldb]; answer b row r at
// out[r * o_ldr + b * o_ldb].
struct BatchIO {
    const uint32_t* Q;
    uint64_t q_ldj, q_ldb;
    uint32_t* out;
    uint64_t o_ldr, o_ldb;
};

// Limb planes of a batch (the matrix-core path's B operand): row n holds
// one limb of one query, entries byte ^ 0x80 as int8, zero-padded to Cp
// columns, stored in 4 KiB tiles of 32 rows x 128 bytes, tile (n/32, k/128)
// at ((n/32) Cp/128 + k/128) 4096.  Byte offset of element (n, 0), and the
// offset added for column k.  Wide layout: row (b/32) 128 + 32 limb + b%32
// for query b.
__device__ inline uint64_t ql_row(uint32_t n, uint32_t Cp) {
    return (uint64_t)(n / 32u) * 32u * Cp + (uint64_t)(n % 32u) * 128u;
}
__device__ inline uint32_t ql_col(uint32_t k) { return (k >> 7) * 4096u + (k & 127u); }

// ---- single-query path (answer_gemv.hip)
uint32_t gemv_variant_count();
const char* gemv_variant_name(uint32_t v);
size_t gemv_workspace_bytes(const pir_db_t* db);
pir_status gemv_answer(const pir_db_t* db, const uint32_t* q, uint32_t* a, void* ws,
                       size_t ws_bytes, hipStream_t s);

// Batches of at most kFewMax queries streamed with dot4 instead of the
// matrix cores (answer_gemv.hip); modulus 0 = mod 2^32, else the field form.
constexpr uint32_t kFewMax = 4;
size_t few_workspace_bytes(const pir_db_t* db, uint32_t B);
pir_status few_answer_batch(const pir_db_t* db, const BatchIO& io, uint32_t B, uint32_t modulus,
                            void* ws, size_t ws_bytes, hipStream_t s);

// ---- database metadata (db.hip)
pir_status launch_rowsum(const pir_db_t* db, const uint32_t* rows, uint32_t m, hipStream_t s);
pir_status launch_scatter_rows(const pir_db_t* db, const uint32_t* rows, uint32_t m,
                               const uint8_t* src, hipStream_t s);

// ---- batched / hint path (answer_mfma.hip)
pir_status mfma_init();
uint32_t mfma_variant_count();
const char* mfma_variant_name(uint32_t v);
bool mfma_variant_valid(const pir_db_t* db, uint32_t B, uint32_t v, bool gathered);
size_t mfma_workspace_bytes(const pir_db_t* db, uint32_t B);
// A batched call's choices (variant, layout, split-K plan) and the
// workspace bytes it touches, all checked before anything is enqueued.
struct BatchPlan {
    uint32_t variant;
    bool few;                    // dot4 stream (answer_gemv.hip)
    uint32_t Bp, N, Cp;          // queries in the limb layout, limb rows, padded columns
    size_t colsum_off, part_off;
    uint32_t M, splits, kts;     // output rows, split-K pieces, k-tiles per piece
    size_t need;                 // workspace bytes the call touches
};
// modulus == 0: Out mod 2^32; otherwise Out mod modulus (field form).
// Returns an error, with nothing enqueued, for calls the kernels cannot serve.
// `planes`: the call will read pre-ingested wide-layout limb planes.
pir_status mfma_plan_batch(const pir_db_t* db, uint32_t B, const uint32_t* rows, uint32_t m,
                           uint32_t modulus, bool planes, BatchPlan* plan);
// Enqueue a planned call; `ws` must hold plan.need bytes, 256-byte aligned;
// `planes` (or null) as written by mfma_ingest_planes for these queries.
pir_status mfma_run_batch(const pir_db_t* db, const BatchIO& io, uint32_t B,
                          const uint32_t* rows, uint32_t modulus, const BatchPlan& plan, void* ws,
                          const void* planes, hipStream_t s);
// Plan, check the workspace against mfma_workspace_bytes (and the planes
// against mfma_planes_bytes), run.
pir_status mfma_answer_batch(const pir_db_t* db, const BatchIO& io, uint32_t B,
                             const uint32_t* rows, uint32_t m, uint32_t modulus, void* ws,
                             size_t ws_bytes, const void* planes, size_t planes_bytes,
                             hipStream_t s);
// Limb planes and column sums of n query columns in the wide layout.
size_t mfma_planes_bytes(const pir_db_t* db, uint32_t n);
pir_status mfma_ingest_planes(const pir_db_t* db, const uint32_t* A, uint32_t n, void* planes,
                              size_t planes_bytes, hipStream_t s);

// ---- allocation-free batched Answer (noalloc.hip)
// Resolve the device address of the fixed scratch array on `dev` (current),
// once per device; later calls return the first outcome.
pir_status noalloc_init_device(int dev);

// ---- XOR (Chor) path (chor.hip)
bool current_is_gfx950();
// out[i] = init[i] (or 0) for i < n (a fill kernel: safe under graph capture).
pir_status chor_init(uint32_t* d_out, const uint32_t* d_init, uint64_t n, hipStream_t s);
// out[b] = init[b] (or 0) xor XOR of the rows of DB selected by query b.
// Arguments already checked by the caller.
pir_status chor_xor(const uint32_t* d_DB, uint32_t rows, uint32_t words, uint64_t pitch,
                    const uint32_t* d_Q, uint32_t B, const uint32_t* d_init, uint32_t* d_out,
                    hipStream_t s);
