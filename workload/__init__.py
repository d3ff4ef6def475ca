"""Seeded synthetic inputs for the LWE-form PIR Answer.

This module is shared by the CPU oracle and the GPU path and therefore holds
only random draws and shapes: no modular products, no query encryption, no
decoding.  Randomness that the LWE client would draw (secret, error, queried
column) is produced here and handed to whichever side builds the query.

Workload recipe (the paper's spectrum databases are synthetic records of
spectrum data, puzzles and signatures; the Answer is a dense, data-oblivious
integer product, so uniform bytes stand in for the records at the same
shapes):

* database ``D``: ``R x C`` uint8, i.i.d. uniform in ``[0, 256)``; rows are
  location-cell x channel records, a record is laid down as one column;
* public matrix ``A``: ``C x n`` uint32, uniform;
* secret ``s``: ``n`` uint32, uniform;
* error ``e``: ``C`` int32 draws of a rounded normal with standard deviation
  ``sigma`` (6.4), tail-cut at ``12 * sigma``;
* queried column ``i``: uniform in ``[0, C)``;
* serving traces: Poisson arrivals at a given rate, database picked by a
  Zipf(s) law over a listed order (rank 1 first).

Host generators use numpy's PCG64.  Databases too large to draw on the host
in reasonable time (gigabytes) are drawn on the device with torch's seeded
generator; tests copy the sampled rows they check back to the host.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 20251003
LWE_N = 1024
LWE_SIGMA = 6.4
LOG_Q = 32          # ciphertext modulus 2^32
LOG_P = 8           # plaintext modulus 2^8 (one database byte)


@dataclasses.dataclass(frozen=True)
class Shape:
    name: str
    rows: int
    cols: int
    batch: int = 1
    n: int = LWE_N


# The five workloads the build is measured and checked on.
CONFIGS = {
    "tiny": Shape("tiny 1024x1024 single query + hint", 1024, 1024, 1),
    "spectrum_1q": Shape("32768x32768 u8 DB, single query", 32768, 32768, 1),
    "spectrum_b64": Shape("32768x32768 u8 DB, 64 queries + hint", 32768, 32768, 64),
    "serving": Shape("8 regional DBs, Poisson 2000 q/s, Zipf(1.1)", 0, 0, 0),
    "large_b256": Shape("131072x131072 u8 DB, 256 queries + 1% row update", 131072, 131072, 256),
}

# Regional database shapes of the serving workload, in Zipf rank order.
SERVING_DBS = [
    (4096, 4096), (8192, 8192), (16384, 8192), (16384, 16384),
    (32768, 16384), (32768, 32768), (65536, 16384), (65536, 32768),
]
SERVING_RATE = 2000.0
SERVING_ZIPF_S = 1.1


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def db_bytes(g: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """Uniform uint8 database, row-major ``rows x cols``."""
    return g.integers(0, 256, size=(rows, cols), dtype=np.uint8)


def uniform_u32(g: np.random.Generator, shape) -> np.ndarray:
    return g.integers(0, 1 << 32, size=shape, dtype=np.uint32)


def lwe_error(g: np.random.Generator, size, sigma: float = LWE_SIGMA) -> np.ndarray:
    """Rounded-normal error draws (standard deviation ``sigma``), int32.

    Draws beyond 12 sigma are redrawn, so every value lies in [-77, 77] for
    sigma = 6.4.
    """
    bound = math.ceil(12 * sigma)
    e = np.rint(g.normal(0.0, sigma, size=size)).astype(np.int64)
    bad = np.abs(e) > bound
    while bad.any():
        e[bad] = np.rint(g.normal(0.0, sigma, size=int(bad.sum()))).astype(np.int64)
        bad = np.abs(e) > bound
    return e.astype(np.int32)


@dataclasses.dataclass
class LweDraws:
    """The client's random draws for ``batch`` queries against ``cols`` columns."""
    s: np.ndarray      # (batch, n) uint32 secrets
    e: np.ndarray      # (batch, cols) int32 errors
    col: np.ndarray    # (batch,) int64 queried columns


def lwe_draws(g: np.random.Generator, cols: int, n: int = LWE_N, batch: int = 1,
              sigma: float = LWE_SIGMA) -> LweDraws:
    s = uniform_u32(g, (batch, n))
    e = lwe_error(g, (batch, cols), sigma)
    col = g.integers(0, cols, size=batch, dtype=np.int64)
    return LweDraws(s=s, e=e, col=col)


def distinct_rows(g: np.random.Generator, rows: int, m: int) -> np.ndarray:
    """``m`` distinct row indices, uniform without replacement, as uint32."""
    return np.sort(g.choice(rows, size=m, replace=False)).astype(np.uint32)


def update_count(rows: int, fraction: float = 0.01) -> int:
    """Rows rewritten by a refresh of ``fraction`` of the database."""
    return int(round(fraction * rows))


def poisson_arrivals(g: np.random.Generator, rate: float, duration_s: float) -> np.ndarray:
    """Open-loop arrival times in seconds, exponential gaps at ``rate`` per second."""
    n_est = int(rate * duration_s * 1.2 + 100)
    t = np.cumsum(g.exponential(1.0 / rate, size=n_est))
    while t[-1] < duration_s:
        more = np.cumsum(g.exponential(1.0 / rate, size=n_est)) + t[-1]
        t = np.concatenate([t, more])
    return t[t < duration_s]


def zipf_probs(k: int, s: float = SERVING_ZIPF_S) -> np.ndarray:
    w = 1.0 / np.arange(1, k + 1, dtype=np.float64) ** s
    return w / w.sum()


def zipf_choice(g: np.random.Generator, k: int, size: int, s: float = SERVING_ZIPF_S) -> np.ndarray:
    return g.choice(k, size=size, p=zipf_probs(k, s)).astype(np.int64)


def device_db(rows: int, cols: int, seed: int, device="cuda"):
    """Uniform uint8 database drawn on ``device`` with torch's seeded generator.

    Used for the gigabyte-scale shapes; the rows a test checks are copied
    back to the host.  Drawn in slabs to bound temporary memory.
    """
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    out = torch.empty((rows, cols), dtype=torch.uint8, device=device)
    slab = max(1, (1 << 28) // max(cols, 1))
    for r0 in range(0, rows, slab):
        r1 = min(rows, r0 + slab)
        out[r0:r1].random_(0, 256, generator=gen)
    return out


def device_u32(shape, seed: int, device="cuda"):
    """Uniform 32-bit words drawn on ``device``, returned as an int32 tensor
    holding the uint32 bit patterns (torch has few uint32 kernels)."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    t = torch.empty(shape, dtype=torch.int64, device=device)
    t.random_(0, 1 << 32, generator=gen)
    t = torch.where(t >= (1 << 31), t - (1 << 32), t)
    return t.to(torch.int32)


# Chor XOR PIR workloads (the ENS instantiation's measurements: databases of
# 2^12 .. 2^18 entries of 3 KB each, batches of 1, 2^7 and 2^10 queries).
CHOR_ENTRY_BYTES = 3072
CHOR_ROWS = (1 << 12, 1 << 14, 1 << 16, 1 << 18)
CHOR_BATCHES = (1, 1 << 7, 1 << 10)


def chor_query_words(g: np.random.Generator, rows: int, batch: int) -> np.ndarray:
    """Uniformly random selector bits, packed 32 per word (batch x ceil(rows/32));
    bits past ``rows`` are zero."""
    nw = (rows + 31) // 32
    q = uniform_u32(g, (batch, nw))
    tail = rows - 32 * (nw - 1)
    if tail < 32:
        q[:, -1] &= np.uint32((1 << tail) - 1)
    return q


def chor_shares(g: np.random.Generator, rows: int, theta: int, servers: int) -> np.ndarray:
    """Random draws of a Chor client: ``servers - 1`` uniform selector words
    per server (the last server's share is fixed by the client from these
    and theta).  Returns (servers - 1) x ceil(rows/32) words."""
    return chor_query_words(g, rows, servers - 1)


# Goldberg IT-PIR (FTR instantiation) workloads: the same database sizes and
# batches as the Chor ones.  The database is stored with one row per byte
# position of a record and one column per record (R = 3072, C = records), so
# a share vector over the records is one query column.  Words are bytes in
# Z/p for the largest prime below 2^32.
FTR_RECORD_BYTES = 3072
FTR_RECORDS = CHOR_ROWS
FTR_BATCHES = CHOR_BATCHES
FTR_PRIME = 4294967291          # 2^32 - 5


def uniform_mod(g: np.random.Generator, shape, p: int) -> np.ndarray:
    """Uniform residues in [0, p) as uint32 (share polynomial coefficients,
    or share-like query words)."""
    return g.integers(0, int(p), size=shape, dtype=np.uint64).astype(np.uint32)


def device_mod(shape, p: int, seed: int, device="cuda"):
    """Uniform residues in [0, p) drawn on ``device``, as an int32 tensor
    holding the uint32 bit patterns."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    t = torch.empty(shape, dtype=torch.int64, device=device)
    t.random_(0, int(p), generator=gen)
    t = torch.where(t >= (1 << 31), t - (1 << 32), t)
    return t.to(torch.int32)
