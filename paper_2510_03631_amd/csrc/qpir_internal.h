// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "qpir.h"

struct pir_db {
    uint32_t magic;        // kDbMagic while open
    uint8_t* D;            // borrowed database bytes
    uint64_t rows, cols, pitch;
    uint32_t* rowterm;     // device, rows words: 0x80808080 * sum_j D[r][j]
    int device;
    bool aligned;          // D and pitch are multiples of 16
};

constexpr uint32_t kDbMagic = 0x51504952u;   // "QPIR"
constexpr uint64_t kMaxDim = (1ull << 31) - 1;
constexpr size_t kWsAlign = 256;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

inline bool db_ok(const pir_db_t* db) { return db && db->magic == kDbMagic; }

inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

#define PIR_LAUNCH_CHECK()                                   \
    do {                                                     \
        if (hipGetLastError() != hipSuccess) return PIR_ERR_DEVICE; \
    } while (0)

// ---- single-query path (answer_gemv.hip)
size_t gemv_workspace_bytes(const pir_db_t* db);
pir_status gemv_answer(const pir_db_t* db, const uint32_t* q, uint32_t* a, void* ws,
                       size_t ws_bytes, hipStream_t s);

// ---- database metadata (db.hip)
pir_status launch_rowterm(const pir_db_t* db, const uint32_t* rows, uint32_t m, hipStream_t s);
pir_status launch_scatter_rows(const pir_db_t* db, const uint32_t* rows, uint32_t m,
                               const uint8_t* src, hipStream_t s);

// ---- batched / hint path (answer_mfma.hip)
size_t mfma_workspace_bytes(const pir_db_t* db, uint32_t B);
pir_status mfma_answer_batch(const pir_db_t* db, const uint32_t* Q, uint32_t B, uint32_t* out,
                             const uint32_t* rows, uint32_t m, void* ws, size_t ws_bytes,
                             hipStream_t s);
