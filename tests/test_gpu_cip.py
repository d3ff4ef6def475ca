"""CIP-PIR (OOP) on the GPU against the oracle, bit for bit: the ChaCha20
expansion, the offline values, the online responses, and the client round
trip over n servers (each server's local database on the device), at small
shapes and at the 2^18-block workload (sampled)."""
import numpy as np
import pytest

import oracle
from oracle import cip
import workload
from _util import banner, to_dev_u32, to_host_u32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qp(gpu):
    import paper_2510_03631_amd as p
    return p


@pytest.mark.parametrize("count,bits", [(1, 1), (3, 31), (2, 32), (5, 33), (7, 1000),
                                        (64, 4096 + 17), (3, 196608)])
def test_prg_expand(qp, count, bits):
    g = np.random.default_rng(count * 1000 + bits)
    seeds = workload.uniform_u32(g, (count, 8))
    banner(f"prg expand count={count} bits={bits}")
    got = to_host_u32(qp.prg_expand(to_dev_u32(seeds), bits))
    exp = np.stack([cip.prg_bits(seeds[e], bits) for e in range(count)])
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("n,t,k,W,count", [(4, 2, 37, 3, 1), (4, 4, 100, 8, 5), (3, 3, 64, 768, 70),
                                           (5, 2, 333, 5, 3), (4, 1, 40, 4, 2), (2, 2, 1000, 12, 130)])
def test_offline_and_answer(qp, n, t, k, W, count):
    g = np.random.default_rng(n * 1000 + t * 100 + k + W + count)
    blocks = workload.uniform_u32(g, (n * k, W))
    i = int(g.integers(0, n))
    loc = cip.server_db(blocks, n, t, i)
    seeds = workload.uniform_u32(g, (count, 8))
    banner(f"oop offline n={n} t={t} k={k} W={W} count={count}")
    A = qp.oop_offline(to_dev_u32(loc), k, t, to_dev_u32(seeds))
    expA = np.stack([cip.offline(loc, k, seeds[e]) for e in range(count)])
    assert np.array_equal(to_host_u32(A), expA)
    Q = workload.chor_query_words(g, k, count)
    banner(f"oop answer n={n} t={t} k={k} W={W} B={count}")
    got = to_host_u32(qp.oop_answer(to_dev_u32(loc), k, to_dev_u32(Q), A))
    exp = np.stack([cip.answer(loc, k, Q[b], expA[b]) for b in range(count)])
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("n,t,k,W", [(4, 4, 256, 768), (3, 2, 77, 6)])
def test_round_trip(qp, n, t, k, W):
    """Several retrievals at once: per retrieval every server pops its own
    (seed, A) pair; the XOR of the servers' GPU responses is the block."""
    import torch
    g = np.random.default_rng(n + t + k + W)
    blocks = workload.uniform_u32(g, (n * k, W))
    thetas = [0, n * k - 1, k, int(g.integers(0, n * k)), int(g.integers(0, n * k))]
    B = len(thetas)
    seeds = workload.uniform_u32(g, (n, B, 8))              # server i, retrieval b
    locs = [to_dev_u32(cip.server_db(blocks, n, t, i)) for i in range(n)]
    A = [qp.oop_offline(locs[i], k, t, to_dev_u32(seeds[i])) for i in range(n)]
    qw = (k + 31) // 32
    Qs = np.zeros((n, B, qw), dtype=np.uint32)
    for b, th in enumerate(thetas):
        Qs[:, b] = cip.client_queries(th, seeds[:, b], n, t, k)
    banner(f"oop round trip n={n} t={t} k={k} W={W} B={B}")
    resp = [to_host_u32(qp.oop_answer(locs[c], k, to_dev_u32(Qs[c]), A[c])) for c in range(n)]
    torch.cuda.synchronize()
    got = cip.reconstruct(resp)
    assert np.array_equal(got, blocks[thetas])


@pytest.mark.parametrize("B", workload.CHOR_BATCHES)
def test_fullsize_sampled(qp, B):
    """2^18 blocks of 3 KB, n = 4 servers each holding every chunk (t = 4),
    as in the benchmark: one server's offline values and online responses,
    sampled entries against the oracle."""
    import torch
    n, t = 4, 4
    r, W = workload.CHOR_ROWS[-1], workload.CHOR_ENTRY_BYTES // 4
    k = r // n
    loc = workload.device_u32((t * k, W), workload.SEED_BASE + 80, "cuda")
    g = workload.rng(workload.SEED_BASE + 81 + B)
    seeds = workload.uniform_u32(g, (B, 8))
    Q = workload.chor_query_words(g, k, B)
    banner(f"oop full size r={r} W={W} B={B}")
    A = qp.oop_offline(loc, k, t, to_dev_u32(seeds))
    out = qp.oop_answer(loc, k, to_dev_u32(Q), A)
    torch.cuda.synchronize()
    host = loc.cpu().numpy().view(np.uint32)
    Ah, outh = to_host_u32(A), to_host_u32(out)
    for b in sorted({0, B - 1, int(g.integers(0, B))}):
        expA = cip.offline(host, k, seeds[b])
        assert np.array_equal(Ah[b], expA), b
        assert np.array_equal(outh[b], cip.answer(host, k, Q[b], expA)), b


def test_error_paths(qp):
    import torch
    from paper_2510_03631_amd._lib import lib
    INVALID_ARG, SHAPE, WORKSPACE = 1, 2, 6
    banner("oop error paths")
    loc = torch.zeros((8, 4), dtype=torch.int32, device="cuda")
    seeds = torch.zeros((2, 8), dtype=torch.int32, device="cuda")
    A = torch.zeros((2, 4), dtype=torch.int32, device="cuda")
    L = lib()
    assert L.pir_prg_expand(seeds.data_ptr(), 2, 0, A.data_ptr(), None) == INVALID_ARG
    assert L.pir_prg_expand(None, 2, 8, A.data_ptr(), None) == INVALID_ARG
    assert L.pir_prg_expand(seeds.data_ptr(), 0, 8, None, None) == 0          # no-op
    # k = 0, pitch < words
    assert L.pir_oop_offline(loc.data_ptr(), 0, 2, 4, 4, seeds.data_ptr(), 2, A.data_ptr(),
                             None, 0, None) == SHAPE
    assert L.pir_oop_answer(loc.data_ptr(), 4, 4, 3, seeds.data_ptr(), 2, A.data_ptr(),
                            A.data_ptr(), None) == SHAPE
    # missing workspace (t = 2 needs the expanded bits)
    assert L.pir_oop_offline(loc.data_ptr(), 4, 2, 4, 4, seeds.data_ptr(), 2, A.data_ptr(),
                             None, 0, None) == WORKSPACE
    torch.cuda.synchronize()
    assert not A.any()
