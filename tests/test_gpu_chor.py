"""Chor XOR PIR on the GPU against the oracle (bit-exact)."""
import numpy as np
import pytest

import oracle
import workload
from _util import banner, to_dev_u32, to_host_u32

pytestmark = pytest.mark.gpu
M32 = 1 << 32


@pytest.fixture(scope="module")
def qp(gpu):
    import paper_2510_03631_amd as p
    return p


@pytest.mark.parametrize("rows,W", [(1, 1), (31, 3), (32, 4), (33, 768), (100, 5),
                                    (1000, 1025), (4097, 12)])
@pytest.mark.parametrize("B", [1, 3, 5, 16, 17, 40, 100, 150, 200, 300, 512, 700])
def test_chor_ragged(qp, rows, W, B):
    banner(f"chor rows={rows} W={W} B={B}")
    g = np.random.default_rng(rows * 7 + W * 3 + B)
    DB = g.integers(0, M32, size=(rows, W), dtype=np.uint32)
    Q = workload.chor_query_words(g, rows, B)
    got = to_host_u32(qp.chor_answer(to_dev_u32(DB), to_dev_u32(Q)))
    assert np.array_equal(got, oracle.chor_answer_batch(DB, Q))


def test_chor_padded_pitch_and_junk_padding_bits(qp):
    import torch
    banner("chor padded pitch, set padding bits")
    g = np.random.default_rng(2)
    rows, W, B = 70, 9, 3
    DB = g.integers(0, M32, size=(rows, W), dtype=np.uint32)
    store = torch.zeros((rows, W + 3), dtype=torch.int32, device="cuda")
    store[:, :W] = to_dev_u32(DB)
    Q = workload.chor_query_words(g, rows, B)
    Qj = Q.copy()
    Qj[:, -1] |= np.uint32(0xFFFFFFFF) << np.uint32(rows % 32)   # bits past the last row
    got = to_host_u32(qp.chor_answer(store[:, :W], to_dev_u32(Qj)))
    assert np.array_equal(got, oracle.chor_answer_batch(DB, Q))


def test_chor_reconstruction_on_device(qp):
    banner("chor 3-server reconstruction")
    g = np.random.default_rng(9)
    rows, W, theta = 5000, 768, 4321
    DB = g.integers(0, M32, size=(rows, W), dtype=np.uint32)
    shares = list(workload.chor_shares(g, rows, theta, 3))
    e = np.zeros(rows, dtype=bool)
    e[theta] = True
    last = oracle.chor_pack(e)
    for s in shares:
        last = last ^ s
    Q = np.stack(shares + [last])
    resp = to_host_u32(qp.chor_answer(to_dev_u32(DB), to_dev_u32(Q)))
    assert np.array_equal(resp[0] ^ resp[1] ^ resp[2], DB[theta])


@pytest.mark.parametrize("B", [1, 128, 200, 1024])
def test_chor_paper_scale(qp, B):
    """2^18 entries of 3 KB (768 MiB), batches of 1, 2^7 and 2^10 queries."""
    banner(f"chor 2^18 x 3KB, B={B}")
    rows, W = 1 << 18, workload.CHOR_ENTRY_BYTES // 4
    DB_d = workload.device_u32((rows, W), workload.SEED_BASE + 60, "cuda")
    DB = DB_d.cpu().numpy().view(np.uint32)
    g = workload.rng(workload.SEED_BASE + 61 + B)
    Q = workload.chor_query_words(g, rows, B)
    out = to_host_u32(qp.chor_answer(DB_d, to_dev_u32(Q)))
    for b in sorted(set([0, B - 1, B // 2])):
        assert np.array_equal(out[b], oracle.chor_answer(DB, Q[b])), b
    # GF(2) Freivalds: the XOR of a random subset of responses equals the
    # response to the XOR of those queries (linearity of the XOR product).
    for t in range(6 if B > 1 else 0):
        pick = g.random(B) < 0.5
        if not pick.any():
            continue
        qx = np.bitwise_xor.reduce(Q[pick], axis=0)
        assert np.array_equal(np.bitwise_xor.reduce(out[pick], axis=0),
                              oracle.chor_answer(DB, qx)), t
