// C ABI entry points: argument checks, handle lifecycle and dispatch.
#include <string.h>

#include <mutex>
#include <new>

#include "qpir_internal.h"

namespace {

bool device_is_gfx950(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
    return strncmp(prop.gcnArchName, "gfx950", 6) == 0;
}

pir_status init_once() {
    static std::once_flag once;
    static pir_status st = PIR_OK;
    std::call_once(once, [] { st = mfma_init(); });
    return st;
}

// Calls must run with the handle's device current.
bool on_db_device(const pir_db_t* db) {
    int dev = -1;
    return hipGetDevice(&dev) == hipSuccess && dev == db->device;
}

}  // namespace

extern "C" {

const char* pir_status_string(pir_status status) {
    switch (status) {
        case PIR_OK: return "ok";
        case PIR_ERR_INVALID_ARG: return "invalid argument";
        case PIR_ERR_SHAPE: return "shape out of range";
        case PIR_ERR_NO_MEMORY: return "out of memory";
        case PIR_ERR_DEVICE: return "device error";
        case PIR_ERR_UNSUPPORTED:
            return "unsupported (gfx950 required, or no kernel serves this layout or variant)";
        case PIR_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
        case PIR_ERR_BUSY: return "queue full";
        case PIR_ERR_TIMEOUT: return "timed out";
    }
    return "unknown status";
}

uint32_t pir_version(void) { return (1u << 16) | 1u; }

pir_status pir_db_open(uint8_t* d_D, uint64_t rows, uint64_t cols, uint64_t row_pitch,
                       pir_stream_t stream, pir_db_t** out) {
    if (!d_D || !out) return PIR_ERR_INVALID_ARG;
    if (rows == 0 || cols == 0 || rows > kMaxDim || cols > kMaxDim || row_pitch < cols)
        return PIR_ERR_SHAPE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return PIR_ERR_DEVICE;
    if (!device_is_gfx950(dev)) return PIR_ERR_UNSUPPORTED;
    if (init_once() != PIR_OK) return PIR_ERR_DEVICE;
    (void)noalloc_init_device(dev);   // its outcome matters only to pir_answer_batch_noalloc

    pir_db_t* db = new (std::nothrow) pir_db_t();
    if (!db) return PIR_ERR_NO_MEMORY;
    db->D = d_D;
    db->rows = rows;
    db->cols = cols;
    db->pitch = row_pitch;
    db->device = dev;
    db->aligned = ((uintptr_t)d_D % 16 == 0) && (row_pitch % 16 == 0);
    for (auto& slot : db->split_rows) slot.store(0, std::memory_order_relaxed);
    if (hipMalloc(&db->rowsum, rows * sizeof(uint32_t)) != hipSuccess) {
        delete db;
        return PIR_ERR_NO_MEMORY;
    }
    db->magic = kDbMagic;
    hipStream_t s = static_cast<hipStream_t>(stream);
    pir_status st = launch_rowsum(db, nullptr, (uint32_t)rows, s);
    if (st == PIR_OK && hipStreamSynchronize(s) != hipSuccess) st = PIR_ERR_DEVICE;
    if (st != PIR_OK) {
        db->magic = 0;
        (void)hipFree(db->rowsum);
        delete db;
        return st;
    }
    *out = db;
    return PIR_OK;
}

pir_status pir_db_close(pir_db_t* db) {
    if (!db) return PIR_OK;
    if (!db_ok(db)) return PIR_ERR_INVALID_ARG;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(db->device);
    pir_status st = PIR_OK;
    if (hipDeviceSynchronize() != hipSuccess) st = PIR_ERR_DEVICE;
    if (hipFree(db->rowsum) != hipSuccess) st = PIR_ERR_DEVICE;
    if (prev >= 0) (void)hipSetDevice(prev);
    db->magic = 0;
    delete db;
    return st;
}

pir_status pir_db_shape(const pir_db_t* db, uint64_t* rows, uint64_t* cols) {
    if (!db_ok(db) || !rows || !cols) return PIR_ERR_INVALID_ARG;
    *rows = db->rows;
    *cols = db->cols;
    return PIR_OK;
}

size_t pir_workspace_bytes(const pir_db_t* db, uint32_t batch) {
    if (!db_ok(db)) return 0;
    return batch == 0 ? gemv_workspace_bytes(db) : mfma_workspace_bytes(db, batch);
}

pir_status pir_answer(pir_db_t* db, const uint32_t* d_q, uint32_t* d_a, void* d_ws,
                      size_t ws_bytes, pir_stream_t stream) {
    if (!db_ok(db) || !d_q || !d_a) return PIR_ERR_INVALID_ARG;
    if (!on_db_device(db)) return PIR_ERR_INVALID_ARG;
    return gemv_answer(db, d_q, d_a, d_ws, ws_bytes, static_cast<hipStream_t>(stream));
}

pir_status pir_answer_batch(pir_db_t* db, const uint32_t* d_Q, uint32_t B, uint32_t* d_out,
                            void* d_ws, size_t ws_bytes, pir_stream_t stream) {
    if (!db_ok(db)) return PIR_ERR_INVALID_ARG;
    if (B == 0) return PIR_OK;
    if (!d_Q || !d_out || !on_db_device(db)) return PIR_ERR_INVALID_ARG;
    if (B > kMaxBatch) return PIR_ERR_SHAPE;
    const BatchIO io{d_Q, B, 1, d_out, B, 1};
    return mfma_answer_batch(db, io, B, nullptr, 0, 0, d_ws, ws_bytes, nullptr, 0,
                             static_cast<hipStream_t>(stream));
}

pir_status pir_answer_batch_qmajor(pir_db_t* db, const uint32_t* d_Qt, uint32_t B,
                                   uint32_t* d_outT, void* d_ws, size_t ws_bytes,
                                   pir_stream_t stream) {
    if (!db_ok(db)) return PIR_ERR_INVALID_ARG;
    if (B == 0) return PIR_OK;
    if (!d_Qt || !d_outT || !on_db_device(db)) return PIR_ERR_INVALID_ARG;
    if (B > kMaxBatch) return PIR_ERR_SHAPE;
    const BatchIO io{d_Qt, 1, db->cols, d_outT, 1, db->rows};
    return mfma_answer_batch(db, io, B, nullptr, 0, 0, d_ws, ws_bytes, nullptr, 0,
                             static_cast<hipStream_t>(stream));
}

pir_status pir_answer_batch_modp(pir_db_t* db, const uint32_t* d_Q, uint32_t B, uint32_t p,
                                 uint32_t* d_out, void* d_ws, size_t ws_bytes,
                                 pir_stream_t stream) {
    if (!db_ok(db) || p < 2) return PIR_ERR_INVALID_ARG;
    if (B == 0) return PIR_OK;
    if (!d_Q || !d_out || !on_db_device(db)) return PIR_ERR_INVALID_ARG;
    if (B > kMaxBatch) return PIR_ERR_SHAPE;
    const BatchIO io{d_Q, B, 1, d_out, B, 1};
    return mfma_answer_batch(db, io, B, nullptr, 0, p, d_ws, ws_bytes, nullptr, 0,
                             static_cast<hipStream_t>(stream));
}

pir_status pir_setup_hint(pir_db_t* db, const uint32_t* d_A, uint32_t n, uint32_t* d_H,
                          void* d_ws, size_t ws_bytes, pir_stream_t stream) {
    if (!db_ok(db) || !d_A || !d_H || n == 0 || !on_db_device(db)) return PIR_ERR_INVALID_ARG;
    if (n > kMaxBatch) return PIR_ERR_SHAPE;
    const BatchIO io{d_A, n, 1, d_H, n, 1};
    return mfma_answer_batch(db, io, n, nullptr, 0, 0, d_ws, ws_bytes, nullptr, 0,
                             static_cast<hipStream_t>(stream));
}

pir_status pir_update_rows(pir_db_t* db, const uint32_t* d_rows, uint32_t m,
                           const uint8_t* d_new, pir_stream_t stream) {
    if (!db_ok(db)) return PIR_ERR_INVALID_ARG;
    if (m == 0) return PIR_OK;
    if (!d_rows || !d_new || !on_db_device(db)) return PIR_ERR_INVALID_ARG;
    if (m > db->rows) return PIR_ERR_SHAPE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    pir_status st = launch_scatter_rows(db, d_rows, m, d_new, s);
    if (st != PIR_OK) return st;
    return launch_rowsum(db, d_rows, m, s);
}

pir_status pir_hint_update_rows(pir_db_t* db, const uint32_t* d_rows, uint32_t m,
                                const uint32_t* d_A, uint32_t n, uint32_t* d_H, void* d_ws,
                                size_t ws_bytes, pir_stream_t stream) {
    if (!db_ok(db)) return PIR_ERR_INVALID_ARG;
    if (m == 0) return PIR_OK;
    if (!d_rows || !d_A || !d_H || n == 0 || !on_db_device(db)) return PIR_ERR_INVALID_ARG;
    if (m > db->rows) return PIR_ERR_SHAPE;
    if (n > kMaxBatch) return PIR_ERR_SHAPE;
    const BatchIO io{d_A, n, 1, d_H, n, 1};
    return mfma_answer_batch(db, io, n, d_rows, m, 0, d_ws, ws_bytes, nullptr, 0,
                             static_cast<hipStream_t>(stream));
}

size_t pir_hint_planes_bytes(const pir_db_t* db, uint32_t n) {
    if (!db_ok(db) || n > kMaxBatch) return 0;
    return mfma_planes_bytes(db, n);
}

pir_status pir_hint_planes(pir_db_t* db, const uint32_t* d_A, uint32_t n, void* d_planes,
                           size_t planes_bytes, pir_stream_t stream) {
    if (!db_ok(db) || !d_A || n == 0 || !on_db_device(db)) return PIR_ERR_INVALID_ARG;
    if (n > kMaxBatch) return PIR_ERR_SHAPE;
    return mfma_ingest_planes(db, d_A, n, d_planes, planes_bytes,
                              static_cast<hipStream_t>(stream));
}

pir_status pir_hint_update_rows_planes(pir_db_t* db, const uint32_t* d_rows, uint32_t m,
                                       const void* d_planes, size_t planes_bytes, uint32_t n,
                                       uint32_t* d_H, void* d_ws, size_t ws_bytes,
                                       pir_stream_t stream) {
    if (!db_ok(db)) return PIR_ERR_INVALID_ARG;
    if (m == 0) return PIR_OK;
    if (!d_rows || !d_planes || !d_H || n == 0 || !on_db_device(db)) return PIR_ERR_INVALID_ARG;
    if (m > db->rows) return PIR_ERR_SHAPE;
    if (n > kMaxBatch) return PIR_ERR_SHAPE;
    const BatchIO io{nullptr, n, 1, d_H, n, 1};
    return mfma_answer_batch(db, io, n, d_rows, m, 0, d_ws, ws_bytes, d_planes, planes_bytes,
                             static_cast<hipStream_t>(stream));
}

uint32_t pir_variant_count(uint32_t batch) {
    return batch == 0 ? gemv_variant_count() : mfma_variant_count();
}

const char* pir_variant_name(uint32_t batch, uint32_t variant) {
    const char* n = batch == 0 ? gemv_variant_name(variant) : mfma_variant_name(variant);
    return n ? n : "invalid";
}

pir_status pir_db_set_variant(pir_db_t* db, uint32_t batch, uint32_t variant) {
    if (!db_ok(db)) return PIR_ERR_INVALID_ARG;
    const bool gathered = (batch & PIR_VARIANT_ROWS) != 0;
    batch &= ~PIR_VARIANT_ROWS;
    if (batch > kMaxBatch) return PIR_ERR_SHAPE;
    if (gathered && batch == 0) return PIR_ERR_INVALID_ARG;
    if (batch == 0) {
        if (variant >= gemv_variant_count()) return PIR_ERR_INVALID_ARG;
    } else {
        if (variant >= mfma_variant_count()) return PIR_ERR_INVALID_ARG;
        if (!mfma_variant_valid(db, batch, variant, gathered)) return PIR_ERR_UNSUPPORTED;
    }
    (gathered ? db->variant_rows : db->variant)[batch_bucket(batch)] = (uint8_t)variant;
    return PIR_OK;
}

uint32_t pir_db_get_variant(const pir_db_t* db, uint32_t batch) {
    const bool gathered = (batch & PIR_VARIANT_ROWS) != 0;
    batch &= ~PIR_VARIANT_ROWS;
    if (!db_ok(db) || batch > kMaxBatch || (gathered && batch == 0)) return 0;
    return (gathered ? db->variant_rows : db->variant)[batch_bucket(batch)];
}

}  // extern "C"
