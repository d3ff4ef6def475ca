/*
 * qpir.h -- C ABI of the MI355X (gfx950) PIR Answer library.
 *
 * The library computes the server side of single-server LWE private
 * information retrieval over a byte database held in GPU memory:
 *
 *   answer      a   = D q        mod 2^32   (D: R x C bytes, q: C words)
 *   batch       Out = D Q        mod 2^32   (Q: C x B words)
 *   hint        H   = D A        mod 2^32   (A: C x n words, offline)
 *   field       Out = D Q        mod p      (Goldberg shares, p < 2^32)
 *   xor         out = XOR of the rows a bit vector selects (Chor, CIP-PIR)
 *
 * This is the response step of the PIR interface (Definition 1: each
 * database server turns a query into a response derived from its local
 * database), its multi-request form (the batched responses of Section 5.2,
 * Algorithms 3 and 4), and the offline/online split of Section 5.3 (the
 * client-independent product D A is computed ahead of the online phase).
 * The paper admits any post-quantum PIR in place of its three
 * instantiations (Section 5.1); this library provides the LWE-based one,
 * whose response is a plain matrix-vector product modulo 2^32.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Pointers prefixed d_ are DEVICE pointers on the device that was current
 *   at pir_db_open.  The caller owns every buffer; the library neither frees
 *   nor retains them after the call returns, except the database bytes that
 *   a handle borrows (see pir_db_open).
 * - Matrices are row-major, elements of 32-bit words are unsigned and all
 *   arithmetic wraps modulo 2^32 (results are exact, bit for bit), except
 *   pir_answer_batch_modp, which reduces the exact product modulo p.
 * - Work is enqueued on `stream` (a hipStream_t; NULL is the null stream)
 *   and the call returns without waiting; results are valid once the stream
 *   reaches that point.  Only pir_db_open and pir_db_close synchronize.
 * - Arguments are checked before anything is enqueued.  On any error the
 *   call returns a status other than PIR_OK and enqueues nothing, so outputs
 *   are left untouched.  No call prints, aborts or throws.
 * - Calls that take a workspace (d_ws, ws_bytes) use it as scratch device
 *   memory of at least pir_workspace_bytes(...) bytes, 256-byte aligned; the
 *   library allocates no device memory on these paths, so they can be
 *   captured into a HIP graph.  Concurrent calls must not share a workspace.
 */
#ifndef QPIR_H
#define QPIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pir_status {
    PIR_OK = 0,
    PIR_ERR_INVALID_ARG = 1,   /* null pointer, bad handle, zero size */
    PIR_ERR_SHAPE = 2,         /* sizes that do not fit the handle or limits */
    PIR_ERR_NO_MEMORY = 3,     /* device or host allocation failed */
    PIR_ERR_DEVICE = 4,        /* a HIP call or kernel launch failed */
    PIR_ERR_UNSUPPORTED = 5,   /* device is not gfx950, or no kernel serves this
                                  combination (field form on gathered rows or on
                                  an unaligned database beyond 4 queries, a
                                  variant the database cannot run) */
    PIR_ERR_WORKSPACE = 6,     /* workspace missing, too small or misaligned */
    PIR_ERR_BUSY = 7,          /* serving queue full: request not admitted */
    PIR_ERR_TIMEOUT = 8        /* wait ended before the request completed */
} pir_status;

/* A hipStream_t, passed as an opaque pointer. */
typedef void* pir_stream_t;

/* Opaque database handle. */
typedef struct pir_db pir_db_t;

/* Static description of a status code; never NULL. */
const char* pir_status_string(pir_status status);

/* Library ABI version, (major << 16) | minor. */
uint32_t pir_version(void);

/*
 * Open a handle on a database resident in device memory (the database is
 * kept in GPU memory for its lifetime, Section 7: no per-query transfers).
 *
 *   d_D        R x C bytes; row r starts at d_D + r * row_pitch.  BORROWED:
 *              the caller keeps the memory alive and unchanged (except
 *              through pir_update_rows) until pir_db_close.
 *   rows, cols R >= 1, C >= 1, both < 2^31.
 *   row_pitch  bytes between row starts, >= cols.  The fast paths need
 *              d_D and row_pitch to be multiples of 16; other values are
 *              served by slower, equally exact kernels.
 *   stream     stream for the metadata pass (per-row byte sums, R words of
 *              device memory allocated and owned by the handle).  The call
 *              synchronizes this stream before returning.
 *   out        receives the handle.
 *
 * Errors: PIR_ERR_INVALID_ARG (null d_D or out), PIR_ERR_SHAPE (sizes),
 * PIR_ERR_UNSUPPORTED (current device is not gfx950), PIR_ERR_NO_MEMORY,
 * PIR_ERR_DEVICE.
 */
pir_status pir_db_open(uint8_t* d_D, uint64_t rows, uint64_t cols, uint64_t row_pitch,
                       pir_stream_t stream, pir_db_t** out);

/* Release the handle and its metadata.  Synchronizes the device first so no
 * queued work still reads the metadata.  NULL is accepted (no-op). */
pir_status pir_db_close(pir_db_t* db);

/* Shape of an open handle. */
pir_status pir_db_shape(const pir_db_t* db, uint64_t* rows, uint64_t* cols);

/*
 * Workspace bytes needed by a call on `db`:
 *   batch == 0   pir_answer
 *   batch == B   pir_answer_batch, pir_answer_batch_qmajor and
 *                pir_answer_batch_modp with B queries, pir_setup_hint and
 *                pir_hint_update_rows with n = B.
 * The value may be 0.
 */
size_t pir_workspace_bytes(const pir_db_t* db, uint32_t batch);

/*
 * Single-query Answer: a[r] = sum_j D[r][j] * q[j] mod 2^32  (Definition 1,
 * response step; one request of Algorithm 3/4's batch).
 *
 *   d_q   C words (the query).  16-byte alignment enables the fast path.
 *   d_a   R words (the answer).  Must not overlap d_q or the database.
 *   d_ws  workspace of pir_workspace_bytes(db, 0) bytes (NULL allowed when
 *         that is 0).
 */
pir_status pir_answer(pir_db_t* db, const uint32_t* d_q, uint32_t* d_a,
                      void* d_ws, size_t ws_bytes, pir_stream_t stream);

/*
 * Batched Answer: Out[r][b] = sum_j D[r][j] * Q[j][b] mod 2^32 for B
 * independent queries (the multi-request response of Section 5.2).  Column b
 * is bit-identical to pir_answer on Q[:, b].  B == 0 is a no-op (PIR_OK).
 *
 *   d_Q    C x B words, row-major (query b is column b).
 *   d_out  R x B words, row-major.
 *   d_ws   workspace of pir_workspace_bytes(db, B) bytes.
 */
pir_status pir_answer_batch(pir_db_t* db, const uint32_t* d_Q, uint32_t B, uint32_t* d_out,
                            void* d_ws, size_t ws_bytes, pir_stream_t stream);

/*
 * Allocation-free batched Answer, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same operands, kernels and results as
 * pir_answer_batch (column b bit-identical to pir_answer on Q[:, b]), but
 * without a workspace argument: the limb planes, column sums and split-K
 * partials go to a fixed array of PIR_NOALLOC_SCRATCH_BYTES of device
 * memory that the library holds on each device it runs on until the
 * process ends.  The call allocates nothing.
 *
 *   d_Q    C x B words, row-major.   d_out  R x B words, row-major.
 *
 * Every call on one device shares that device's array: calls that overlap
 * on a device (other streams, other threads, other handles) race and give
 * undefined results; the caller orders them (one stream, or events).  The
 * array keeps the last call's contents; each call rewrites what it reads.
 * Errors: as pir_answer_batch, and PIR_ERR_SHAPE (nothing enqueued) when
 * the call needs more than PIR_NOALLOC_SCRATCH_BYTES of scratch (about
 * 4 * B * C bytes of limb planes plus the split-K partials; 64 queries fit
 * a 32768 x 32768 database), PIR_ERR_DEVICE when the array's address could
 * not be resolved on this device.
 */
#define PIR_NOALLOC_SCRATCH_BYTES (64u << 20)
pir_status pir_answer_batch_noalloc(pir_db_t* db, const uint32_t* d_Q, uint32_t B,
                                    uint32_t* d_out, pir_stream_t stream);

/*
 * Batched Answer in query-major layout: query b is the contiguous row
 * Qt[b][0..C) and its answer the contiguous row outT[b][0..R), i.e.
 * outT[b][r] = sum_j D[r][j] * Qt[b][j] mod 2^32.  Same kernels and results
 * as pir_answer_batch; the layout lets a server pack and unpack individual
 * queries with plain copies.
 *
 *   d_Qt    B x C words, row-major.   d_outT  B x R words, row-major.
 *   d_ws    workspace of pir_workspace_bytes(db, B) bytes.
 */
pir_status pir_answer_batch_qmajor(pir_db_t* db, const uint32_t* d_Qt, uint32_t B,
                                   uint32_t* d_outT, void* d_ws, size_t ws_bytes,
                                   pir_stream_t stream);

/*
 * Batched Answer over a prime field: Out[r][b] = sum_j D[r][j] * Q[j][b]
 * mod p.  This is the server product of the Goldberg (FTR) instantiation
 * (Section 5.1; the "mod q" batched product of Algorithm 4): each query
 * column holds one server's Shamir shares (one field element per database
 * column), and the client interpolates the servers' responses.  Database
 * bytes are field elements in [0, 256); query words are taken as integers
 * (normally residues in [0, p)); the result is exact, reduced once.
 *
 *   p      modulus, 2 <= p < 2^32 (prime for Shamir sharing; not checked).
 *   d_Q    C x B words, row-major.   d_out  R x B words in [0, p), row-major.
 *   d_ws   workspace of pir_workspace_bytes(db, B) bytes.
 * Requires a 16-byte aligned database with C a multiple of 16
 * (PIR_ERR_UNSUPPORTED otherwise) and C <= 2^23 (PIR_ERR_SHAPE).  p < 2
 * gives PIR_ERR_INVALID_ARG.  B == 0 is a no-op.
 */
pir_status pir_answer_batch_modp(pir_db_t* db, const uint32_t* d_Q, uint32_t B, uint32_t p,
                                 uint32_t* d_out, void* d_ws, size_t ws_bytes,
                                 pir_stream_t stream);

/*
 * Offline hint: H = D A mod 2^32 (the client-independent part of the
 * response, moved off the online path as in Section 5.3).
 *
 *   d_A   C x n words, row-major (the public LWE matrix).
 *   d_H   R x n words, row-major.
 *   d_ws  workspace of pir_workspace_bytes(db, n) bytes.
 */
pir_status pir_setup_hint(pir_db_t* db, const uint32_t* d_A, uint32_t n, uint32_t* d_H,
                          void* d_ws, size_t ws_bytes, pir_stream_t stream);

/*
 * Database refresh (records are rewritten each validity interval, Section
 * 4.2): D[rows[i]][:] = new[i][:] for i < m, and the handle's per-row
 * metadata is updated to match.
 *
 *   d_rows  m DISTINCT row indices < R (device).  Indices >= R are skipped;
 *           duplicate indices leave the affected rows unspecified.
 *   d_new   m x C bytes, row-major, tightly packed.
 *   The caller orders this call after every queued answer on the database
 *   (same stream, or an event) -- it writes the borrowed bytes.
 */
pir_status pir_update_rows(pir_db_t* db, const uint32_t* d_rows, uint32_t m,
                           const uint8_t* d_new, pir_stream_t stream);

/*
 * Incremental hint after a refresh: H[rows[i]][:] = D[rows[i]][:] A mod 2^32
 * for i < m; every other row of H is left as it is.  Equal to a full
 * pir_setup_hint on the refreshed database, at the cost of m rows.
 *
 *   d_rows  as for pir_update_rows.
 *   d_A     C x n words; d_H R x n words.
 *   d_ws    workspace of pir_workspace_bytes(db, n) bytes.
 */
pir_status pir_hint_update_rows(pir_db_t* db, const uint32_t* d_rows, uint32_t m,
                                const uint32_t* d_A, uint32_t n, uint32_t* d_H,
                                void* d_ws, size_t ws_bytes, pir_stream_t stream);

/*
 * The incremental hint from limb planes of A prepared once.  A is fixed for
 * a deployment (the public LWE matrix), while rows are refreshed every
 * validity interval (Section 4.2); pir_hint_update_rows re-derives A's
 * 8-bit limb planes on every call, and these entry points let a caller
 * derive them once (the offline work of Section 5.3 kept off the refresh
 * path).
 *
 * pir_hint_planes_bytes: bytes of the prepared planes of n columns of A for
 *   databases with this handle's column count (0 for a bad handle).
 * pir_hint_planes: write them.
 *   d_A      C x n words, row-major (as for pir_setup_hint).
 *   d_planes device buffer of pir_hint_planes_bytes(db, n) bytes, 256-byte
 *            aligned, caller-owned; its content is opaque and stays valid
 *            for any handle with the same column count until A changes.
 * pir_hint_update_rows_planes: pir_hint_update_rows with A given by its
 *   prepared planes (same results, bit for bit).
 *   d_planes, planes_bytes  as written by pir_hint_planes for this n.
 *   d_ws     workspace of pir_workspace_bytes(db, n) bytes.
 * Errors: PIR_ERR_INVALID_ARG (null pointer, n == 0), PIR_ERR_SHAPE,
 * PIR_ERR_WORKSPACE (planes or workspace missing, too small or misaligned).
 */
size_t pir_hint_planes_bytes(const pir_db_t* db, uint32_t n);
pir_status pir_hint_planes(pir_db_t* db, const uint32_t* d_A, uint32_t n, void* d_planes,
                           size_t planes_bytes, pir_stream_t stream);
pir_status pir_hint_update_rows_planes(pir_db_t* db, const uint32_t* d_rows, uint32_t m,
                                       const void* d_planes, size_t planes_bytes, uint32_t n,
                                       uint32_t* d_H, void* d_ws, size_t ws_bytes,
                                       pir_stream_t stream);

/*
 * Client side of LWE PIR on the GPU (Definition 1: the client builds the
 * queries and reconstructs the block from the responses), for B queries at
 * once.  No handle needed; runs on the current device (gfx950).
 *
 * pir_client_query:   Qt[b][j] = sum_k A[j][k] S[b][k] + E[b][j]
 *                                + (j == cols[b] ? 2^24 : 0)      mod 2^32
 *   d_A     C x n words (the public matrix), row-major.
 *   d_S     B x n words (secrets); d_E  B x C signed errors; d_cols B indices.
 *   d_Qt    B x C words: query b is row b (the layout of
 *           pir_answer_batch_qmajor, and of pir_answer for B == 1).
 *
 * pir_client_decode:  out[b][r] = ((answers[b][r] - sum_k H[r][k] S[b][k]
 *                                   + 2^23) mod 2^32) >> 24
 *   d_H     R x n words (the hint), row-major.
 *   d_answers  B x R words; d_out  B x R bytes (the recovered column).
 *
 * Errors: PIR_ERR_INVALID_ARG (null pointer), PIR_ERR_SHAPE (zero or
 * oversized dimension), PIR_ERR_UNSUPPORTED (device not gfx950).
 */
pir_status pir_client_query(const uint32_t* d_A, uint32_t C, uint32_t n, const uint32_t* d_S,
                            const int32_t* d_E, const uint32_t* d_cols, uint32_t B,
                            uint32_t* d_Qt, pir_stream_t stream);
pir_status pir_client_decode(const uint32_t* d_H, uint32_t R, uint32_t n, const uint32_t* d_S,
                             const uint32_t* d_answers, uint32_t B, uint8_t* d_out,
                             pir_stream_t stream);

/*
 * The same client steps on the matrix cores, for batches of secrets.  Over
 * Z/2^32 a word matrix is the sum of its byte planes, M = sum_i 2^(8i) M_i,
 * so M x = [M_0 | M_1 | M_2 | M_3] [x; 2^8 x; 2^16 x; 2^24 x]: a byte matrix
 * times a word vector, the Answer product itself.  A prepared client matrix
 * holds those byte planes (the public matrix A for queries, the hint H for
 * decoding) and a batch of B secrets runs through the batched Answer, then
 * the query or decode epilogue.  Results are bit-identical to
 * pir_client_query / pir_client_decode.
 *
 * pir_client_mat_open: prepare M (rows x n words, row-major, device; read
 *   during the call only).  Allocates rows x 4n bytes of device memory and a
 *   database handle over them, owned by the returned object; synchronizes
 *   `stream`.  Errors: PIR_ERR_INVALID_ARG, PIR_ERR_SHAPE,
 *   PIR_ERR_UNSUPPORTED, PIR_ERR_NO_MEMORY, PIR_ERR_DEVICE.
 * pir_client_mat_close: release it (synchronizes the device; NULL is a no-op).
 * pir_client_mat_workspace_bytes: workspace of a batch of B secrets, for
 *   either call (0 for a bad handle or B).
 * The secrets' operand goes straight into the product's limb layout (one
 * kernel), so a call is that kernel, the product and the epilogue.
 * pir_client_query_mat: pir_client_query with A prepared: S, E, cols and Qt
 *   as there, C = rows.
 * pir_client_decode_mat: pir_client_decode with H prepared: S, answers and
 *   out as there, R = rows.
 *   d_ws  workspace of pir_client_mat_workspace_bytes(M, B) bytes, 256-byte
 *         aligned (PIR_ERR_WORKSPACE otherwise).
 */
typedef struct pir_client_mat pir_client_mat_t;
pir_status pir_client_mat_open(const uint32_t* d_M, uint32_t rows, uint32_t n,
                               pir_stream_t stream, pir_client_mat_t** out);
pir_status pir_client_mat_close(pir_client_mat_t* mat);
size_t pir_client_mat_workspace_bytes(const pir_client_mat_t* mat, uint32_t B);
/* Kernel variant of the product for batches in B's bucket (as
 * pir_db_set_variant; for the autotuner). */
pir_status pir_client_mat_set_variant(pir_client_mat_t* mat, uint32_t batch, uint32_t variant);
pir_status pir_client_query_mat(pir_client_mat_t* A, const uint32_t* d_S, const int32_t* d_E,
                                const uint32_t* d_cols, uint32_t B, uint32_t* d_Qt, void* d_ws,
                                size_t ws_bytes, pir_stream_t stream);
pir_status pir_client_decode_mat(pir_client_mat_t* H, const uint32_t* d_S,
                                 const uint32_t* d_answers, uint32_t B, uint8_t* d_out,
                                 void* d_ws, size_t ws_bytes, pir_stream_t stream);

/*
 * Chor XOR PIR response (the ENS instantiation, Section 5.1; the server step
 * of Algorithm 3), for B queries:
 *     out[b] = XOR of the rows i of DB whose bit i is set in query b.
 *
 *   d_DB    rows x words 32-bit words (a row is one b-bit block), row i at
 *           d_DB + i * row_pitch_words.  16-byte alignment with words and
 *           row_pitch_words multiples of 4 enables the vector path.
 *   d_Q     B x ceil(rows / 32) words: query b packed 32 rows per word,
 *           bit j of word k selecting row 32k + j; bits past the last row
 *           are ignored.
 *   d_out   B x words (cleared and written by the call).
 *   B == 0 is a no-op.  Errors: PIR_ERR_INVALID_ARG, PIR_ERR_SHAPE,
 *   PIR_ERR_UNSUPPORTED.
 */
pir_status pir_chor_answer(const uint32_t* d_DB, uint32_t rows, uint32_t words,
                           uint64_t row_pitch_words, const uint32_t* d_Q, uint32_t B,
                           uint32_t* d_out, pir_stream_t stream);

/*
 * CIP-PIR, the OOP instantiation (Section 5.1: full instantiation; proof of
 * Lemma 2).  The database's r blocks form n chunks of k blocks; server i
 * stores t of them, chunk i (its flip chunk) first, then chunks i+1 ..
 * i+t-1 mod n (non-flip).  A server's local database is therefore t*k rows
 * of `words` 32-bit words (the layout of pir_chor_answer), rows 0 .. k-1
 * being the flip chunk.
 *
 * pir_prg_expand: the PRG.  For each of `count` 8-word seeds, the first
 *   `bits` bits of the ChaCha20 keystream (RFC 8439 block function; seed =
 *   key, nonce 0, block counter from 0), as ceil(bits/32) words per seed
 *   (keystream words in order, little endian; bits past `bits` cleared).
 *     d_seeds  count x 8 words.   d_out  count x ceil(bits/32) words.
 *
 * pir_oop_offline: the client-independent precomputation.  For each seed e,
 *   A[e] = XOR of the non-flip rows k + m (m < k(t-1)) whose bit m is set in
 *   pir_prg_expand(seed e, k(t-1)).  t == 1 gives A = 0.
 *     d_DB     the server's local database (t*k rows).
 *     d_A      count x words.
 *     d_ws     pir_oop_workspace_bytes(k, t, count) bytes, 256-byte aligned
 *              (NULL allowed when that is 0): the expanded selector bits.
 *
 * pir_oop_answer: the online response.  For each query b,
 *   out[b] = A[b] xor (XOR of the flip-chunk rows i < k whose bit i is set
 *   in query b), with queries packed as for pir_chor_answer over k rows.
 *     d_Q  B x ceil(k/32) words.   d_A, d_out  B x words (d_A[b] is the
 *     offline value paired with query b's seed).
 *
 * count == 0 or B == 0 is a no-op.  Errors: PIR_ERR_INVALID_ARG (null
 * pointer, bits == 0), PIR_ERR_SHAPE (zero or oversized sizes, pitch <
 * words), PIR_ERR_WORKSPACE, PIR_ERR_UNSUPPORTED (device not gfx950).
 */
pir_status pir_prg_expand(const uint32_t* d_seeds, uint32_t count, uint32_t bits,
                          uint32_t* d_out, pir_stream_t stream);
size_t pir_oop_workspace_bytes(uint32_t k, uint32_t t, uint32_t count);
pir_status pir_oop_offline(const uint32_t* d_DB, uint32_t k, uint32_t t, uint32_t words,
                           uint64_t row_pitch_words, const uint32_t* d_seeds, uint32_t count,
                           uint32_t* d_A, void* d_ws, size_t ws_bytes, pir_stream_t stream);
pir_status pir_oop_answer(const uint32_t* d_DB, uint32_t k, uint32_t words,
                          uint64_t row_pitch_words, const uint32_t* d_Q, uint32_t B,
                          const uint32_t* d_A, uint32_t* d_out, pir_stream_t stream);

/*
 * Kernel variants (tile shapes, pipeline depths, rows per wave) for the
 * autotuner.  `batch` == 0 names the single-query path, `batch` >= 1 the
 * batched path.  Variant 0 is the library's built-in choice.  Every variant
 * computes the same exact result; only speed differs.
 */
uint32_t pir_variant_count(uint32_t batch);
/* Static name of a variant ("invalid" when out of range); never NULL. */
const char* pir_variant_name(uint32_t batch, uint32_t variant);
/*
 * Use `variant` for calls on `db` whose batch size falls in the same
 * power-of-two bucket as `batch` (batch == 0: pir_answer).  Returns
 * PIR_ERR_UNSUPPORTED when the variant cannot serve that bucket on this
 * database (e.g. a pipelined kernel on an unaligned database), leaving the
 * previous choice in place.  Not synchronized with calls in flight on other
 * threads.
 */
pir_status pir_db_set_variant(pir_db_t* db, uint32_t batch, uint32_t variant);
uint32_t pir_db_get_variant(const pir_db_t* db, uint32_t batch);
/*
 * OR'ed into `batch` (>= 1) of pir_db_set_variant and pir_db_get_variant,
 * selects the table of the row-gathered products (pir_hint_update_rows, with
 * n in that bucket) instead of the whole-database one.  Scattered rows cost
 * address-translation latency, so the two favour different pipelines and
 * are tuned apart; a gathered call with no choice of its own takes the
 * built-in choice for gathered rows.  The single-query path has no gathered
 * form: batch == PIR_VARIANT_ROWS is PIR_ERR_INVALID_ARG.
 */
#define PIR_VARIANT_ROWS 0x80000000u

/*
 * Serving loop: continuous batching of queries over resident databases
 * (the batched, latency-oriented response of Section 5.2).  Host-side
 * queues feed per-database slots (stream, pinned staging, device buffers);
 * a scheduler thread launches whatever has queued whenever a slot is free
 * (and fewer than max_inflight batches have kernels pending), the database
 * with the longest-waiting request first, as one HIP-graph replay per batch
 * (sizes rounded up to powers of two) followed by the copy-out of its
 * answers, and admits a batch only if its device bytes fit the memory
 * budget next to the batches already in flight.
 * Latency runs from the request's (scheduled) arrival time to its answer
 * being in the caller's host buffer.
 */
typedef struct pir_server pir_server_t;

typedef struct pir_server_config {
    uint32_t max_batch;         /* largest batch per launch: power of two, 1..1024 */
    uint32_t slots_per_db;      /* batches in flight per database, 1..16 */
    uint64_t mem_budget_bytes;  /* device bytes of all batches in flight (queries,
                                   answers, workspace), > 0.  It gates launches; it
                                   does not bound what pir_server_start allocates
                                   (every slot holds buffers for max_batch queries
                                   and a workspace for the largest batch; see
                                   pir_server_stats.device_bytes) */
    uint32_t max_queue;         /* queued requests per database before submit
                                   returns PIR_ERR_BUSY; 0 = unbounded */
    uint32_t use_graphs;        /* 1: replay captured HIP graphs; 0: direct launches */
    uint32_t max_inflight;      /* batches with kernels pending, over all databases
                                   (one copying its answers out no longer counts);
                                   0 = only the slots bound them.  A cap keeps requests
                                   queued while the device is busy, so they leave in
                                   larger batches under load */
} pir_server_config;

typedef struct pir_server_stats {
    uint64_t submitted, completed, failed, rejected;
    uint64_t batches, batched_queries;           /* launched batches and their queries */
    uint64_t budget_bytes, peak_inflight_bytes;  /* admission budget and its high-water mark */
    uint64_t p50_ns, p99_ns, max_ns;             /* latency of completed requests */
    uint64_t device_bytes;                       /* device memory the slots hold */
} pir_server_stats;

/* Create a server on the current device (no threads yet). */
pir_status pir_server_create(const pir_server_config* cfg, pir_server_t** out);
/* Register an open database (borrowed; keep it open until destroy).  Only
 * before pir_server_start.  *db_index receives its index. */
pir_status pir_server_add_db(pir_server_t* server, pir_db_t* db, uint32_t* db_index);
/* Allocate slots, capture the graphs and start the scheduler and completion
 * threads.  PIR_ERR_NO_MEMORY if a single query of some database does not
 * fit the budget or an allocation fails.  While batches are in flight the
 * completion thread polls them, yielding between polls, for up to 2 ms after
 * the last completion (then every 20 us), so it keeps one host core busy
 * under load; with nothing in flight it sleeps. */
pir_status pir_server_start(pir_server_t* server);
/*
 * Queue one query (C words, host memory) for database `db_index`.  The
 * answer (R words) is copied to `h_answer` (host; NULL discards it) when the
 * request completes.  Both buffers must stay valid until then.
 * `t_arrival_ns` is the arrival time on pir_server_now_ns()'s clock (0 =
 * now).  *ticket identifies the request.  PIR_ERR_BUSY if the queue is full.
 */
pir_status pir_server_submit(pir_server_t* server, uint32_t db_index, const uint32_t* h_q,
                             uint32_t* h_answer, uint64_t t_arrival_ns, uint64_t* ticket);
/* Monotonic clock used for arrival times, nanoseconds. */
uint64_t pir_server_now_ns(void);
/* Block until the request completes (PIR_OK), fails (PIR_ERR_DEVICE) or
 * `timeout_ns` passes (PIR_ERR_TIMEOUT; UINT64_MAX waits forever). */
pir_status pir_server_wait(pir_server_t* server, uint64_t ticket, uint64_t timeout_ns);
/* Block until every submitted request has completed or failed (PIR_OK, or
 * PIR_ERR_DEVICE if any failed).  Requests queued for a paused database wait
 * for its resume, so while one is held the call returns PIR_ERR_BUSY instead
 * of blocking; the held requests stay queued. */
pir_status pir_server_drain(pir_server_t* server);
/* Stop launching batches for one database and wait for its batches in
 * flight, e.g. around pir_update_rows / pir_hint_update_rows; queued
 * requests wait.  pir_server_resume_db restarts it. */
pir_status pir_server_pause_db(pir_server_t* server, uint32_t db_index);
pir_status pir_server_resume_db(pir_server_t* server, uint32_t db_index);
/* Counters and latency percentiles so far. */
pir_status pir_server_stats_get(pir_server_t* server, pir_server_stats* out);
/* Latencies (ns; 0 = not completed) of tickets first .. first+count-1. */
pir_status pir_server_latencies(pir_server_t* server, uint64_t first, uint64_t count,
                                uint64_t* out_ns);
/*
 * Open-loop load generator: submit request i at offsets_ns[i] after the
 * call starts (scheduled time = arrival time), for database db_index[i],
 * query h_q[i] and answer buffer h_answer[i] (h_answer may be NULL).
 * Returns after the last submission; *first_ticket is the first accepted
 * ticket (UINT64_MAX if none).  Rejected (queue full) requests are counted
 * in the stats and skipped.
 */
pir_status pir_server_replay(pir_server_t* server, uint64_t n, const uint64_t* offsets_ns,
                             const uint32_t* db_index, const uint32_t* const* h_q,
                             uint32_t* const* h_answer, uint64_t* first_ticket);
/* Finish every queued and running request (paused databases are resumed
 * for it), stop the threads and free the server's buffers (not the
 * databases). */
pir_status pir_server_destroy(pir_server_t* server);

#ifdef __cplusplus
}
#endif

#endif /* QPIR_H */
