"""CPU oracle for CIP-PIR, the OOP instantiation -- TEST INFRASTRUCTURE ONLY.

Follows the paper's description of the QPADL-OOP workflow (Section 5.1, the
full instantiation, and the proof of Lemma 2):

* The database holds r blocks; it is cut into n chunks of k = r / n
  consecutive blocks, chunk_c = blocks c*k .. c*k + k - 1.  Server i stores
  t chunks in the order chunk_i, chunk_{i+1}, ..., chunk_{i+t-1} (indices
  mod n); its first chunk is its flip chunk, the other t - 1 are non-flip.
* Offline, server i draws a seed S, expands it with a PRG into k(t-1) bits
  (one per non-flip block, in local order) and stores A = XOR of the
  non-flip blocks whose bit is set, keeping (S, A) for one future query.
* The client, holding every server's seed, starts from the r-bit unit
  vector e_theta, XORs each server's expanded bits into the positions of
  that server's non-flip blocks, and sends server c the k bits of chunk c.
* Server c answers R_c = A_c xor (XOR of the flip-chunk blocks its k bits
  select).  The XOR of all n responses is block theta: every PRG bit is
  added twice (once into the query, once into A) and cancels.

The PRG is ChaCha20 (RFC 8439): the 32-byte seed is the key, the nonce is
zero and the block counter starts at 0; the keystream's 32-bit words (little
endian) are the query words, bit j of word w selecting local non-flip block
32 w + j.  The paper asks only for a secure PRG; ChaCha20 is the choice made
here, pinned against OpenSSL's implementation in the tests.

Blocks are b-bit values stored as W 32-bit words; queries are packed 32
selector bits per word exactly as for Chor PIR (see ``oracle.chor_*``).
"""
from __future__ import annotations

import numpy as np

from . import chor_answer, chor_reconstruct

_MASK = 0xFFFFFFFF
_SIGMA = (0x61707865, 0x3320646E, 0x79622D32, 0x6B206574)   # "expand 32-byte k"


def _rotl(x: np.ndarray, n: int) -> np.ndarray:
    return ((x << np.uint32(n)) | (x >> np.uint32(32 - n))).astype(np.uint32)


def _quarter(s, a, b, c, d):
    s[a] = s[a] + s[b]; s[d] = _rotl(s[d] ^ s[a], 16)
    s[c] = s[c] + s[d]; s[b] = _rotl(s[b] ^ s[c], 12)
    s[a] = s[a] + s[b]; s[d] = _rotl(s[d] ^ s[a], 8)
    s[c] = s[c] + s[d]; s[b] = _rotl(s[b] ^ s[c], 7)


def chacha20_blocks(key, counters, nonce=(0, 0, 0)) -> np.ndarray:
    """ChaCha20 block function for each counter: returns len(counters) x 16
    words.  key: 8 words, nonce: 3 words (RFC 8439, Section 2.3)."""
    key = [int(k) & _MASK for k in key]
    counters = np.asarray(counters, dtype=np.uint32)
    m = counters.size
    init = np.empty((16, m), dtype=np.uint32)
    init[0:4] = np.array(_SIGMA, dtype=np.uint32)[:, None]
    init[4:12] = np.array(key, dtype=np.uint32)[:, None]
    init[12] = counters
    init[13:16] = np.array([int(x) & _MASK for x in nonce], dtype=np.uint32)[:, None]
    s = init.copy()
    with np.errstate(over="ignore"):
        for _ in range(10):              # 20 rounds: column round + diagonal round
            _quarter(s, 0, 4, 8, 12)
            _quarter(s, 1, 5, 9, 13)
            _quarter(s, 2, 6, 10, 14)
            _quarter(s, 3, 7, 11, 15)
            _quarter(s, 0, 5, 10, 15)
            _quarter(s, 1, 6, 11, 12)
            _quarter(s, 2, 7, 8, 13)
            _quarter(s, 3, 4, 9, 14)
        out = (s + init).astype(np.uint32)
    return out.T.copy()


def prg_words(seed, nwords: int) -> np.ndarray:
    """First ``nwords`` keystream words of ChaCha20 keyed by the 8-word seed."""
    nblk = (nwords + 15) // 16
    if nblk == 0:
        return np.zeros(0, dtype=np.uint32)
    return chacha20_blocks(seed, np.arange(nblk, dtype=np.uint32)).reshape(-1)[:nwords]


def prg_bits(seed, nbits: int) -> np.ndarray:
    """The PRG's ``nbits``-bit output packed into ceil(nbits/32) words; bits
    past ``nbits`` are zero."""
    nw = (nbits + 31) // 32
    w = prg_words(seed, nw)
    tail = nbits - 32 * (nw - 1) if nw else 32
    if nw and tail < 32:
        w[-1] &= np.uint32((1 << tail) - 1)
    return w


def server_db(blocks: np.ndarray, n: int, t: int, i: int) -> np.ndarray:
    """Local database of server i: chunks i, i+1, ..., i+t-1 (mod n) of the
    r x W block matrix, in that order (t*k x W words)."""
    r = blocks.shape[0]
    assert r % n == 0 and 1 <= t <= n
    k = r // n
    return np.concatenate([blocks[((i + c) % n) * k:((i + c) % n + 1) * k] for c in range(t)])


def offline(local: np.ndarray, k: int, seed) -> np.ndarray:
    """A = XOR of the non-flip blocks (local rows k .. t*k - 1) selected by
    the PRG expansion of ``seed`` (k(t-1) bits)."""
    nonflip = local[k:]
    return chor_answer(nonflip, prg_bits(seed, nonflip.shape[0]))


def answer(local: np.ndarray, k: int, qwords, A) -> np.ndarray:
    """Online response: A xor (XOR of the flip-chunk blocks the k-bit
    sub-query selects)."""
    return chor_answer(local[:k], qwords) ^ np.asarray(A, dtype=np.uint32)


def client_queries(theta: int, seeds, n: int, t: int, k: int) -> np.ndarray:
    """The n sub-queries (n x ceil(k/32) packed words) for block ``theta``
    given every server's seed (seeds[i] is server i's 8-word seed)."""
    r = n * k
    q = np.zeros(r, dtype=bool)
    q[theta] = True
    for i in range(n):
        v = prg_bits(seeds[i], k * (t - 1))
        bits = ((v[:, None] >> np.arange(32, dtype=np.uint32)) & 1).reshape(-1)[:k * (t - 1)]
        for m in np.nonzero(bits)[0]:
            c = (i + 1 + m // k) % n           # global chunk of local non-flip block m
            q[c * k + m % k] ^= True
    out = np.zeros((n, (k + 31) // 32), dtype=np.uint32)
    for c in range(n):
        sel = q[c * k:(c + 1) * k]
        padded = np.zeros(out.shape[1] * 32, dtype=np.uint32)
        padded[:k] = sel
        out[c] = (padded.reshape(-1, 32) << np.arange(32, dtype=np.uint32)).sum(axis=1)
    return out


def reconstruct(responses) -> np.ndarray:
    """The client's block: XOR of the n responses."""
    return chor_reconstruct(responses)
