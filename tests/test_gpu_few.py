"""The small-batch stream (batches of at most 4 queries, both forms) against
the oracle: ragged and unaligned shapes, column splits for short databases,
both query layouts, and agreement with the matrix-core variants."""
import numpy as np
import pytest

import oracle
import workload
from _util import banner, to_dev_u32, to_dev_u8, to_host_u32

pytestmark = pytest.mark.gpu
P = workload.FTR_PRIME


@pytest.fixture(scope="module")
def qp(gpu):
    import paper_2510_03631_amd as p
    return p


def _unaligned(D):
    import torch
    R, C = D.shape
    store = torch.zeros(R * C + 3, dtype=torch.uint8, device="cuda")
    store[3:] = torch.from_numpy(np.ascontiguousarray(D).reshape(-1)).cuda()
    return store[3:].view(R, C)


@pytest.mark.parametrize("R,C", [(1, 1), (7, 333), (64, 4096), (300, 5000), (2, 65536 + 48),
                                 (1000, 1024)])
@pytest.mark.parametrize("B", [1, 2, 3, 4])
@pytest.mark.parametrize("aligned", [True, False])
def test_few_ring_and_field(qp, R, C, B, aligned):
    g = np.random.default_rng(R * 13 + C + B * 7 + aligned)
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    Q = workload.uniform_u32(g, (C, B))
    Dd = to_dev_u8(D) if aligned else _unaligned(D)
    banner(f"few R={R} C={C} B={B} aligned={aligned}")
    with qp.Database(Dd) as db:
        db.set_variant(B, "few")
        got = to_host_u32(db.answer_batch(to_dev_u32(Q)))
        assert np.array_equal(got, oracle.answer_batch(D, Q))
        got_t = to_host_u32(db.answer_batch_qmajor(to_dev_u32(np.ascontiguousarray(Q.T))))
        assert np.array_equal(got_t, oracle.answer_batch(D, Q).T)
        for p in (65537, P):
            got = to_host_u32(db.answer_batch_modp(to_dev_u32(Q), p))
            assert np.array_equal(got, oracle.answer_batch_mod(D, Q, p)), p


def test_few_extremes_and_default(qp):
    # All-0xFF database against all-ones words: the largest exact sums.
    R, C = 130, 70000
    D = np.full((R, C), 255, dtype=np.uint8)
    Q = np.full((C, 2), 0xFFFFFFFF, dtype=np.uint32)
    banner("few extremes")
    with qp.Database(to_dev_u8(D)) as db:
        assert db.get_variant(2) == 0                      # built-in choice: the stream
        got = to_host_u32(db.answer_batch(to_dev_u32(Q)))
        assert np.array_equal(got, oracle.answer_batch(D, Q))
        got = to_host_u32(db.answer_batch_modp(to_dev_u32(Q), P))
        assert np.array_equal(got, oracle.answer_batch_mod(D, Q, P))


def test_few_matches_matrix_cores(qp):
    R, C = 2048, 8192
    g = np.random.default_rng(3)
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    with qp.Database(to_dev_u8(D)) as db:
        for B in (1, 2, 4):
            Q = to_dev_u32(workload.uniform_u32(g, (C, B)))
            db.set_variant(B, "few")
            a = to_host_u32(db.answer_batch(Q))
            fa = to_host_u32(db.answer_batch_modp(Q, P))
            for name in ("ring_128x128_k128_s4", "reg_128x128"):
                banner(f"few vs {name} B={B}")
                db.set_variant(B, name)
                assert np.array_equal(to_host_u32(db.answer_batch(Q)), a), name
            db.set_variant(B, "ring_128x128_k128_s4")
            assert np.array_equal(to_host_u32(db.answer_batch_modp(Q, P)), fa)
