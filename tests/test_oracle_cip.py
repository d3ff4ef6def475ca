"""Pins of the CIP-PIR (OOP) oracle, CPU only.

* The PRG (ChaCha20) against OpenSSL's ChaCha20 stream cipher, an
  independent library implementation (keystream = encryption of zeros).
* Closed forms of the protocol: the XOR of all servers' responses is the
  requested block for every n, t, theta; without a target bit the responses
  cancel to zero; the offline value A equals a Python-integer XOR of the
  selected non-flip blocks; sub-queries of chunks other than theta's do not
  depend on theta.
"""
import ctypes
import ctypes.util

import numpy as np
import pytest

import oracle
from oracle import cip
import workload


def _openssl():
    for name in ("libcrypto.so.3", ctypes.util.find_library("crypto")):
        if not name:
            continue
        try:
            lib = ctypes.CDLL(name)
            lib.EVP_chacha20.restype = ctypes.c_void_p
            lib.EVP_CIPHER_CTX_new.restype = ctypes.c_void_p
            lib.EVP_EncryptInit_ex.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_char_p, ctypes.c_char_p]
            lib.EVP_EncryptUpdate.argtypes = [ctypes.c_void_p, ctypes.c_char_p,
                                              ctypes.POINTER(ctypes.c_int), ctypes.c_char_p,
                                              ctypes.c_int]
            lib.EVP_CIPHER_CTX_free.argtypes = [ctypes.c_void_p]
            return lib
        except (OSError, AttributeError):
            continue
    return None


def _openssl_keystream(lib, key_words, counter, nbytes):
    key = np.asarray(key_words, dtype="<u4").tobytes()
    iv = np.array([counter, 0, 0, 0], dtype="<u4").tobytes()   # counter || 96-bit nonce 0
    ctx = lib.EVP_CIPHER_CTX_new()
    try:
        assert lib.EVP_EncryptInit_ex(ctx, lib.EVP_chacha20(), None, key, iv) == 1
        out = ctypes.create_string_buffer(nbytes)
        outl = ctypes.c_int(0)
        assert lib.EVP_EncryptUpdate(ctx, out, ctypes.byref(outl), bytes(nbytes), nbytes) == 1
        assert outl.value == nbytes
        return np.frombuffer(out.raw, dtype="<u4").astype(np.uint32)
    finally:
        lib.EVP_CIPHER_CTX_free(ctx)


@pytest.mark.parametrize("seed", range(4))
def test_chacha20_matches_openssl(seed):
    lib = _openssl()
    if lib is None:
        pytest.skip("OpenSSL libcrypto not available to pin ChaCha20 against")
    g = np.random.default_rng(seed)
    key = workload.uniform_u32(g, 8)
    if seed == 0:
        key[:] = 0
    nwords = 16 * 37 + 5
    assert np.array_equal(cip.prg_words(key, nwords), _openssl_keystream(lib, key, 0, 4 * nwords))
    # A later block counter, straight from the block function.
    blk = cip.chacha20_blocks(key, [9])[0]
    assert np.array_equal(blk, _openssl_keystream(lib, key, 9, 64))


def test_prg_bits_packing():
    key = np.arange(8, dtype=np.uint32)
    w = cip.prg_words(key, 4)
    for nbits, nw in ((1, 1), (32, 1), (33, 2), (100, 4)):
        b = cip.prg_bits(key, nbits)
        assert b.size == nw
        assert np.array_equal(b[:-1], w[:nw - 1])
        tail = nbits - 32 * (nw - 1)
        mask = (1 << tail) - 1 if tail < 32 else 0xFFFFFFFF
        assert int(b[-1]) == int(w[nw - 1]) & mask


def test_server_db_layout():
    r, W, n = 12, 3, 4
    blocks = np.arange(r * W, dtype=np.uint32).reshape(r, W)
    k = r // n
    for i in range(n):
        for t in range(1, n + 1):
            loc = cip.server_db(blocks, n, t, i)
            assert loc.shape == (t * k, W)
            for c in range(t):
                g = (i + c) % n
                assert np.array_equal(loc[c * k:(c + 1) * k], blocks[g * k:(g + 1) * k])


def _brute_xor(rows_words, bits):
    acc = 0
    for row, bit in zip(rows_words, bits):
        if bit:
            acc ^= int.from_bytes(np.asarray(row, dtype="<u4").tobytes(), "little")
    return acc


@pytest.mark.parametrize("n,t,k,W", [(2, 2, 37, 3), (3, 2, 64, 2), (4, 4, 33, 5), (5, 3, 40, 1),
                                     (4, 1, 16, 2)])
def test_round_trip_recovers_block(n, t, k, W):
    g = np.random.default_rng(n * 100 + t * 10 + k)
    r = n * k
    blocks = workload.uniform_u32(g, (r, W))
    locs = [cip.server_db(blocks, n, t, i) for i in range(n)]
    for theta in (0, r - 1, k - 1, k, int(g.integers(0, r))):
        seeds = workload.uniform_u32(g, (n, 8))
        A = [cip.offline(locs[i], k, seeds[i]) for i in range(n)]
        qs = cip.client_queries(theta, seeds, n, t, k)
        resp = [cip.answer(locs[c], k, qs[c], A[c]) for c in range(n)]
        assert np.array_equal(cip.reconstruct(resp), blocks[theta])


def test_offline_value_brute_force():
    g = np.random.default_rng(3)
    n, t, k, W = 3, 3, 45, 4
    blocks = workload.uniform_u32(g, (n * k, W))
    loc = cip.server_db(blocks, n, t, 1)
    seed = workload.uniform_u32(g, 8)
    bits_w = cip.prg_bits(seed, k * (t - 1))
    bits = oracle.chor_unpack(bits_w, k * (t - 1))
    exp = _brute_xor(loc[k:], bits)
    got = cip.offline(loc, k, seed)
    assert int.from_bytes(got.astype("<u4").tobytes(), "little") == exp


def test_masks_cancel_and_other_chunks_ignore_theta():
    g = np.random.default_rng(4)
    n, t, k = 4, 3, 40
    seeds = workload.uniform_u32(g, (n, 8))
    q1 = cip.client_queries(5, seeds, n, t, k)          # theta in chunk 0
    q2 = cip.client_queries(17, seeds, n, t, k)         # also chunk 0
    assert np.array_equal(q1[1:], q2[1:])               # other chunks do not see theta
    assert not np.array_equal(q1[0], q2[0])
    # Without the target bit the responses cancel: XOR of (A_c xor masked
    # flip-chunk XOR) over all servers is zero.
    blocks = workload.uniform_u32(g, (n * k, 3))
    locs = [cip.server_db(blocks, n, t, i) for i in range(n)]
    A = [cip.offline(locs[i], k, seeds[i]) for i in range(n)]
    q = q1.copy()
    q[0, 0] ^= np.uint32(1 << 5)                        # remove e_theta
    resp = [cip.answer(locs[c], k, q[c], A[c]) for c in range(n)]
    assert not cip.reconstruct(resp).any()
    # With t >= 2 each sub-query is masked: not the bare unit vector.
    assert int(q1[0][0]) != (1 << 5) or q1[0][1:].any()
