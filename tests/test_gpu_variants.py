"""Every kernel variant the autotuner may pick gives the oracle's exact result."""
import numpy as np
import pytest

import oracle
import workload
from _util import banner, to_dev_u32, to_dev_u8, to_host_u32

pytestmark = pytest.mark.gpu
M32 = 1 << 32


@pytest.fixture(scope="module")
def qp(gpu):
    import paper_2510_03631_amd as p
    return p


@pytest.mark.parametrize("R,C", [(300, 4096), (1000, 1040), (77, 9000), (513, 2048)])
def test_single_query_variants(qp, R, C):
    from paper_2510_03631_amd._lib import variant_names
    g = np.random.default_rng(R + C)
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    q = g.integers(0, M32, size=C, dtype=np.uint32)
    exp = oracle.answer(D, q)
    with qp.Database(to_dev_u8(D)) as db:
        for v, name in enumerate(variant_names(0)):
            banner(f"single variant {name} R={R} C={C}")
            db.set_variant(0, v)
            assert np.array_equal(to_host_u32(db.answer(to_dev_u32(q))), exp), name


@pytest.mark.parametrize("R,C,B", [(300, 4096, 64), (257, 1040, 100), (130, 2000, 7),
                                   (64, 512, 256), (700, 3072, 33), (500, 4096, 3),
                                   (300, 1040, 16), (1000, 2048, 9)])
def test_batch_variants(qp, R, C, B):
    from paper_2510_03631_amd._lib import variant_names
    g = np.random.default_rng(R * 3 + C + B)
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    Q = g.integers(0, M32, size=(C, B), dtype=np.uint32)
    exp = oracle.answer_batch(D, Q)
    tried = 0
    with qp.Database(to_dev_u8(D)) as db:
        for v, name in enumerate(variant_names(B)):
            try:
                db.set_variant(B, v)
            except qp.PirError:
                continue
            banner(f"batch variant {name} R={R} C={C} B={B}")
            assert np.array_equal(to_host_u32(db.answer_batch(to_dev_u32(Q))), exp), name
            Qt = np.ascontiguousarray(Q.T)
            got_t = to_host_u32(db.answer_batch_qmajor(to_dev_u32(Qt)))
            assert np.array_equal(got_t, exp.T), name
            tried += 1
    assert tried >= 3


def test_hint_update_variants(qp):
    from paper_2510_03631_amd._lib import variant_names
    import torch
    g = np.random.default_rng(99)
    R, C, n = 400, 2048, 128
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    A = g.integers(0, M32, size=(C, n), dtype=np.uint32)
    rows = workload.distinct_rows(g, R, 37)
    new = g.integers(0, 256, size=(37, C), dtype=np.uint8)
    D2 = oracle.update_rows(D, rows, new)
    exp = oracle.hint(D2, A)
    for v, name in enumerate(variant_names(n)):
        Dd = to_dev_u8(D)
        with qp.Database(Dd) as db:
            try:
                db.set_variant(n, v)
                db.set_variant(n, v, rows=True)
            except qp.PirError:
                continue
            banner(f"hint update variant {name}")
            Ad = to_dev_u32(A)
            H = db.setup_hint(Ad)
            rd = to_dev_u32(rows)
            db.update_rows(rd, to_dev_u8(new))
            db.hint_update_rows(rd, Ad, H)
            torch.cuda.synchronize()
            assert np.array_equal(to_host_u32(H), exp), name


def test_gathered_variant_table(qp):
    # Row-gathered products keep their own variant table: pinning one table
    # leaves the other alone, the single-query path has no gathered form,
    # and the dot4 'few' kernel (whole database only) is refused for it.
    import torch
    banner("gathered variant table")
    D = torch.zeros((256, 1024), dtype=torch.uint8, device="cuda")
    with qp.Database(D) as db:
        names = qp.variant_names(64)
        db.set_variant(64, "ring_128x128_k128_s4")
        db.set_variant(64, "ring8w_256x256_s4", rows=True)
        assert names[db.get_variant(64)] == "ring_128x128_k128_s4"
        assert names[db.get_variant(64, rows=True)] == "ring8w_256x256_s4"
        db.set_variant(64, 0, rows=True)
        assert db.get_variant(64, rows=True) == 0
        assert names[db.get_variant(64)] == "ring_128x128_k128_s4"
        with pytest.raises(qp.PirError):
            db.set_variant(0, 1, rows=True)
        with pytest.raises(qp.PirError):
            db.set_variant(2, "few", rows=True)
        db.set_variant(2, "few")
        assert db.get_variant(2, rows=True) == 0


def test_unaligned_database_rejects_ring_variants(qp):
    import torch
    banner("unaligned database: ring variants unsupported")
    store = torch.zeros(64 * 100 + 1, dtype=torch.uint8, device="cuda")
    D = store[1:].view(64, 100)
    with qp.Database(D) as db:
        with pytest.raises(qp.PirError):
            db.set_variant(64, "ring_128x256_s6")
        db.set_variant(64, "reg_128x256")
        assert qp.variant_names(64)[db.get_variant(64)] == "reg_128x256"


def test_wide_variants_accumulator_wrap(qp):
    """Every variant that serves 64 queries, on the extremes at C = 131072:
    centred products (-128)(-128) summed to 2^31 wrap the int32
    accumulators; all-0xFF bytes against all-ones words; the answers equal
    the closed form and the oracle."""
    from paper_2510_03631_amd._lib import variant_names
    R, C, B = 300, 131072, 64
    cases = [(0, 0), (255, 0xFFFFFFFF), (0, 0x80808080), (255, 0x7F7F7F7F)]
    tried = set()
    for dval, qval in cases:
        D = np.full((R, C), dval, dtype=np.uint8)
        Q = np.full((C, B), qval, dtype=np.uint32)
        exp = oracle.answer_batch(D, Q)
        assert (exp == (dval * qval * C) % M32).all()
        with qp.Database(to_dev_u8(D)) as db:
            Qd = to_dev_u32(Q)
            for v, name in enumerate(variant_names(B)):
                try:
                    db.set_variant(B, v)
                except qp.PirError:
                    continue
                banner(f"wrap C={C} d={dval} q={qval:#x} {name}")
                assert np.array_equal(to_host_u32(db.answer_batch(Qd)), exp), (name, dval, qval)
                tried.add(name)
    assert len(tried) >= 4
