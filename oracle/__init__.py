"""CPU oracle for the LWE-form PIR Answer -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding)
never calls it and shares no code with it.

Contents
--------
* ``answer`` / ``answer_batch`` / ``hint`` / ``hint_rows``: the server's
  response and offline hint, computed by the plain C loops of
  ``pir_oracle.c`` (built with gcc, OpenMP over output rows).
* ``brute_answer`` / ``brute_answer_batch``: the same definitions summed with
  Python integers and reduced once at the end, for tiny shapes.  They share
  nothing with the C loops and pin them.
* ``lwe_query`` / ``lwe_decode``: the client side of single-server LWE PIR
  (not printed in the paper, which allows any post-quantum PIR in place of its
  three instantiations; Section 5.1): ``q = A s + e + Delta u_i`` and
  ``round((a - H s) / Delta)`` with ``Delta = 2^32 / 256``.
* ``update_rows``: a database refresh (records are rewritten each validity
  interval, Section 4.2), as plain array assignment.
* ``freivalds``: a randomized whole-matrix check of a claimed product over
  Z/2^32, for shapes too large to recompute.
* ``chor_*``: Chor XOR PIR (the ENS instantiation, Section 5.1, and the
  server step of Algorithm 3): XOR of the selected rows, query packing, and
  the client's reconstruction; ``brute_chor`` with Python integers.
* ``answer_batch_mod`` / ``answer_mod_entries`` / ``brute_answer_batch_mod``:
  the Goldberg (FTR) server product ``D Q mod p`` (Section 5.1; Algorithm 4's
  "mod q"), exact sums reduced once (C loops with 128-bit sums; numpy
  uint64 dot products for sampled entries; Python integers).
* ``shamir_shares`` / ``lagrange_at_zero``: the client side of Goldberg's
  IT-PIR as the paper describes it in its security argument: per database
  column j a random degree-t polynomial f_j with f_j(0) = e_theta[j], server
  i receives (f_1(alpha_i), ..., f_r(alpha_i)); the client interpolates the
  servers' responses at 0.  The random coefficients are inputs.

* ``oracle.cip``: CIP-PIR, the OOP instantiation (Section 5.1, full
  instantiation; proof of Lemma 2): chunk layout per server, ChaCha20 PRG,
  offline seed/value pairs, online flip-chunk response, client queries and
  reconstruction (see that module).

Parity is pinned for every function here (see ``tests/test_oracle_pins.py``
and ``tests/test_oracle_cip.py``):
brute force on tiny inputs, closed forms, a hand-worked example, the LWE
round trip and invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pir_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

DELTA = 1 << 24          # 2^32 / 2^8: scale of the plaintext byte in the ciphertext
HALF_DELTA = 1 << 23


def build(force: bool = False) -> str:
    """Compile ``pir_oracle.c`` into ``liboracle.so`` with gcc -O2 -fopenmp."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c11", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        U = ctypes.c_uint64
        lib.oracle_answer.argtypes = [P, U, U, U, P, P]
        lib.oracle_answer_batch_rows.argtypes = [P, U, U, P, U, P, U, P]
        lib.oracle_matvec_u32.argtypes = [P, U, U, P, P]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_answer_batch_mod.argtypes = [P, U, U, P, U, P, U, ctypes.c_uint32, P]
        lib.oracle_answer_batch_mod.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def _as_db(D: np.ndarray) -> np.ndarray:
    D = np.asarray(D)
    assert D.dtype == np.uint8 and D.ndim == 2
    return np.ascontiguousarray(D)


def _as_u32(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint32))


# --------------------------------------------------------------------------
# Server side: answer, batched answer, hint
# --------------------------------------------------------------------------
def answer(D: np.ndarray, q) -> np.ndarray:
    """``a[r] = sum_j D[r, j] * q[j] mod 2^32`` (the per-query response)."""
    D = _as_db(D)
    q = _as_u32(q)
    R, C = D.shape
    assert q.shape == (C,)
    a = np.empty(R, dtype=np.uint32)
    _load().oracle_answer(_p(D), R, C, C, _p(q), _p(a))
    return a


def answer_batch(D: np.ndarray, Q, rows=None) -> np.ndarray:
    """``out[r, b] = sum_j D[r, j] * Q[j, b] mod 2^32`` for ``Q`` of shape C x B.

    With ``rows`` given, only those database rows are computed (output row i
    belongs to database row ``rows[i]``).
    """
    D = _as_db(D)
    Q = _as_u32(Q)
    R, C = D.shape
    assert Q.ndim == 2 and Q.shape[0] == C
    B = Q.shape[1]
    if rows is None:
        m, rp = R, None
    else:
        rows = np.ascontiguousarray(np.asarray(rows, dtype=np.uint64))
        assert rows.size == 0 or int(rows.max()) < R
        m, rp = rows.size, _p(rows)
    out = np.empty((m, B), dtype=np.uint32)
    if m and B:
        _load().oracle_answer_batch_rows(_p(D), C, C, rp, m, _p(Q), B, _p(out))
    elif m:
        out[:] = 0
    return out


def hint(D: np.ndarray, A, rows=None) -> np.ndarray:
    """Offline hint ``H = D A mod 2^32`` (A is C x n); the client-independent
    part of the response, computed ahead of the online phase (Section 5.3)."""
    return answer_batch(D, A, rows=rows)


def matvec_u32(M, x) -> np.ndarray:
    """``y = M x mod 2^32`` for a word matrix ``M`` (rows x n)."""
    M = _as_u32(M)
    x = _as_u32(x)
    R, n = M.shape
    assert x.shape == (n,)
    y = np.empty(R, dtype=np.uint32)
    _load().oracle_matvec_u32(_p(M), R, n, _p(x), _p(y))
    return y


def update_rows(D: np.ndarray, rows, new_rows: np.ndarray) -> np.ndarray:
    """Database refresh: a copy of ``D`` with ``D[rows[i]] = new_rows[i]``."""
    D2 = np.array(D, dtype=np.uint8, copy=True)
    rows = np.asarray(rows, dtype=np.int64)
    assert len(np.unique(rows)) == rows.size, "rows must be distinct"
    D2[rows] = new_rows
    return D2


# --------------------------------------------------------------------------
# Brute force with Python integers (tiny shapes only)
# --------------------------------------------------------------------------
def brute_answer(D, q) -> list:
    R = len(D)
    out = []
    for r in range(R):
        total = 0
        for j in range(len(q)):
            total += int(D[r][j]) * int(q[j])
        out.append(total % (1 << 32))
    return out


def brute_answer_batch(D, Q) -> list:
    C = len(Q)
    B = len(Q[0]) if C else 0
    return [[sum(int(D[r][j]) * int(Q[j][b]) for j in range(C)) % (1 << 32)
             for b in range(B)] for r in range(len(D))]


# --------------------------------------------------------------------------
# LWE client (query construction and decoding)
# --------------------------------------------------------------------------
def lwe_query(A, s, e, col: int) -> np.ndarray:
    """``q = A s + e + Delta * u_col mod 2^32``.

    A: C x n uint32, s: n uint32, e: C signed errors, col: queried column.
    """
    As = matvec_u32(A, s).astype(np.int64)
    q = As + np.asarray(e, dtype=np.int64)
    q[int(col)] += DELTA
    return (q % (1 << 32)).astype(np.uint32)


def lwe_decode(a, H, s) -> np.ndarray:
    """Recover the queried column: ``m = ((a - H s + Delta/2) mod 2^32) >> 24``.

    Rounds to the nearest multiple of Delta, treating the noise ``D e`` as a
    signed value in [-Delta/2, Delta/2).
    """
    Hs = matvec_u32(H, s).astype(np.int64)
    diff = (np.asarray(a, dtype=np.int64) - Hs + HALF_DELTA) % (1 << 32)
    return (diff >> 24).astype(np.uint8)


# --------------------------------------------------------------------------
# Randomized whole-matrix check
# --------------------------------------------------------------------------
def freivalds(D: np.ndarray, Q, out, trials: int = 16, seed: int = 0) -> bool:
    """Check ``out == D Q mod 2^32`` with Freivalds' test.

    Each trial draws a uniform x in (Z/2^32)^B and compares ``out x`` with
    ``D (Q x)``.  A wrong entry e != 0 survives a trial only if e x_b == 0 for
    the random coordinate, probability at most 1/2; ``trials`` rounds leave
    at most 2^-trials.
    """
    g = np.random.Generator(np.random.PCG64(seed))
    Q = _as_u32(Q)
    out = _as_u32(out)
    B = Q.shape[1]
    for _ in range(trials):
        x = g.integers(0, 1 << 32, size=B, dtype=np.uint32)
        lhs = matvec_u32(out, x)
        rhs = answer(D, matvec_u32(Q, x))
        if not np.array_equal(lhs, rhs):
            return False
    return True


# --------------------------------------------------------------------------
# Chor XOR PIR (the ENS instantiation, Section 5.1; server step of
# Algorithm 3): the response to a query bit vector q is the XOR of the
# database rows whose bit is set.  Rows are b-bit blocks stored as W 32-bit
# words; a query over r rows is packed little-endian into ceil(r/32) words
# (bit j of word k selects row 32k + j).
# --------------------------------------------------------------------------
def chor_unpack(qwords, rows: int) -> np.ndarray:
    """Packed query words -> boolean selector of length ``rows``."""
    w = np.asarray(qwords, dtype=np.uint32)
    bits = (w[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1
    return bits.reshape(-1)[:rows].astype(bool)


def chor_pack(sel) -> np.ndarray:
    sel = np.asarray(sel, dtype=bool)
    n = (sel.size + 31) // 32
    padded = np.zeros(n * 32, dtype=np.uint32)
    padded[:sel.size] = sel
    return (padded.reshape(n, 32) << np.arange(32, dtype=np.uint32)).sum(axis=1).astype(np.uint32)


def chor_answer(DBw: np.ndarray, qwords) -> np.ndarray:
    """XOR of the rows of ``DBw`` (r x W words) selected by the packed query."""
    DBw = np.asarray(DBw, dtype=np.uint32)
    sel = chor_unpack(qwords, DBw.shape[0])
    if not sel.any():
        return np.zeros(DBw.shape[1], dtype=np.uint32)
    return np.bitwise_xor.reduce(DBw[sel], axis=0)


def chor_answer_batch(DBw: np.ndarray, Qwords: np.ndarray) -> np.ndarray:
    """One response per row of ``Qwords`` (B x ceil(r/32) packed queries)."""
    return np.stack([chor_answer(DBw, q) for q in np.asarray(Qwords, dtype=np.uint32)])


def chor_reconstruct(responses) -> np.ndarray:
    """The client's block: XOR of the servers' responses (Definition 1's
    BlockReconst for Chor PIR)."""
    out = np.zeros_like(np.asarray(responses[0], dtype=np.uint32))
    for r in responses:
        out ^= np.asarray(r, dtype=np.uint32)
    return out


def brute_chor(rows_bits: list, qbits: list) -> int:
    """Python-integer brute force: rows as b-bit integers, XOR of selected."""
    acc = 0
    for row, bit in zip(rows_bits, qbits):
        if bit:
            acc ^= row
    return acc


# --------------------------------------------------------------------------
# Goldberg IT-PIR (the FTR instantiation, Section 5.1): database words are
# bytes taken as elements of Z/p for a prime p < 2^32; queries are Shamir
# shares; the server's response is the product over Z/p.
# --------------------------------------------------------------------------
def answer_batch_mod(D: np.ndarray, Q, p: int, rows=None) -> np.ndarray:
    """``out[r, b] = (sum_j D[r, j] * Q[j, b]) mod p`` for ``Q`` of shape C x B."""
    D = _as_db(D)
    Q = _as_u32(Q)
    p = int(p)
    assert 2 <= p < 1 << 32
    R, C = D.shape
    assert Q.ndim == 2 and Q.shape[0] == C
    B = Q.shape[1]
    if rows is None:
        m, rp = R, None
    else:
        rows = np.ascontiguousarray(np.asarray(rows, dtype=np.uint64))
        assert rows.size == 0 or int(rows.max()) < R
        m, rp = rows.size, _p(rows)
    out = np.zeros((m, B), dtype=np.uint32)
    if m and B:
        rc = _load().oracle_answer_batch_mod(_p(D), C, C, rp, m, _p(Q), B, p, _p(out))
        assert rc == 0, "oracle_answer_batch_mod: out of memory"
    return out


def answer_mod_entries(D_rows: np.ndarray, Q_cols: np.ndarray, p: int) -> np.ndarray:
    """Sampled entries of ``D Q mod p``: entry k is ``D_rows[k] . Q_cols[k] mod p``.

    D_rows: K x C bytes, Q_cols: K x C words.  The dot products are formed in
    uint64, exact while C * 255 * (2^32 - 1) < 2^64, i.e. C < 2^24.
    """
    D_rows = np.asarray(D_rows, dtype=np.uint8)
    Q_cols = np.asarray(Q_cols, dtype=np.uint32)
    assert D_rows.shape == Q_cols.shape and D_rows.shape[1] < 1 << 24
    tot = np.einsum("kj,kj->k", D_rows.astype(np.uint64), Q_cols.astype(np.uint64))
    return (tot % np.uint64(p)).astype(np.uint32)


def brute_answer_batch_mod(D, Q, p: int) -> list:
    C = len(Q)
    B = len(Q[0]) if C else 0
    return [[sum(int(D[r][j]) * int(Q[j][b]) for j in range(C)) % p for b in range(B)]
            for r in range(len(D))]


def shamir_shares(secret, coeffs, alphas, p: int) -> np.ndarray:
    """Shares of a vector secret: ``out[i, j] = f_j(alphas[i]) mod p`` with
    ``f_j(x) = secret[j] + sum_{k=1..t} coeffs[k-1, j] x^k``.

    secret: r residues, coeffs: t x r residues (uniform draws), alphas:
    distinct nonzero evaluation points, one per server.  Returns len(alphas)
    x r uint32.
    """
    p = int(p)
    secret = np.asarray(secret, dtype=np.uint64) % np.uint64(p)
    coeffs = np.asarray(coeffs, dtype=np.uint64).reshape(-1, secret.size)
    out = np.empty((len(alphas), secret.size), dtype=np.uint32)
    P = np.uint64(p)
    for i, a in enumerate(alphas):
        acc = secret.copy()
        for k in range(coeffs.shape[0]):
            ak = np.uint64(pow(int(a), k + 1, p))            # alpha^k mod p, < 2^32
            acc = (acc + (coeffs[k] % P) * ak % P) % P       # products < 2^64
        out[i] = acc.astype(np.uint32)
    return out


def lagrange_weights_at_zero(alphas, p: int) -> list:
    """``w_i = prod_{m != i} alpha_m / (alpha_m - alpha_i) mod p``, so that a
    polynomial of degree < len(alphas) has ``f(0) = sum_i w_i f(alpha_i)``."""
    p = int(p)
    al = [int(a) % p for a in alphas]
    w = []
    for i, ai in enumerate(al):
        num, den = 1, 1
        for m, am in enumerate(al):
            if m != i:
                num = num * am % p
                den = den * (am - ai) % p
        w.append(num * pow(den, -1, p) % p)
    return w


def lagrange_at_zero(alphas, responses, p: int) -> np.ndarray:
    """Interpolate the servers' responses at 0: ``sum_i w_i R_i mod p``
    (the client's reconstruction from any t+1 honest responses)."""
    P = np.uint64(int(p))
    w = lagrange_weights_at_zero(alphas, p)
    acc = np.zeros(np.asarray(responses[0]).shape, dtype=np.uint64)
    for wi, Ri in zip(w, responses):
        acc = (acc + np.uint64(wi) * (np.asarray(Ri, dtype=np.uint64) % P) % P) % P
    return acc.astype(np.uint32)
