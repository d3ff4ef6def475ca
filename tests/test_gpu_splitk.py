"""Split-K on the matrix-core path (mod 2^32): shapes whose output tiles
cannot fill the chip (few rows, long rows, gathered rows of an incremental
hint) cut the K range into pieces whose partial products a finishing kernel
adds.  Every case is compared with the oracle element by element, for every
ring variant that can serve the batch."""
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


def _ring_variants(qp, B):
    return [(v, n) for v, n in enumerate(qp.variant_names(B)) if n.startswith(("ring", "narrow"))]


@pytest.mark.parametrize("R,C,B", [(1, 131072, 1), (64, 65536, 64), (100, 32768, 1),
                                   (257, 16384, 200), (5, 8192 + 48, 33), (70, 40960, 8),
                                   (129, 16384 + 16, 16)])
def test_few_rows_long_rows(qp, R, C, B):
    g = np.random.default_rng(R + C + B)
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    Q = workload.uniform_u32(g, (C, B))
    exp = oracle.answer_batch(D, Q)
    with qp.Database(to_dev_u8(D)) as db:
        Qd = to_dev_u32(Q)
        Qtd = to_dev_u32(np.ascontiguousarray(Q.T))
        for v, name in _ring_variants(qp, B):
            try:
                db.set_variant(B, v)
            except qp.PirError:
                continue
            banner(f"split-K R={R} C={C} B={B} {name}")
            assert np.array_equal(to_host_u32(db.answer_batch(Qd)), exp), name
            assert np.array_equal(to_host_u32(db.answer_batch_qmajor(Qtd)), exp.T), name


@pytest.mark.parametrize("m,n", [(1, 256), (37, 256), (300, 256), (37, 5), (300, 16)])
def test_incremental_hint_gathered_rows(qp, m, n):
    import torch
    R, C = 4096, 16384
    g = np.random.default_rng(m)
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    A = workload.uniform_u32(g, (C, n))
    rows = workload.distinct_rows(g, R, m)
    new = g.integers(0, 256, size=(m, C), dtype=np.uint8)
    D2 = oracle.update_rows(D, rows, new)
    exp = oracle.hint(D2, A, rows=rows)
    with qp.Database(to_dev_u8(D)) as db:
        Ad = to_dev_u32(A)
        H = torch.zeros((R, n), dtype=torch.int32, device="cuda")
        rows_d = to_dev_u32(rows)
        db.update_rows(rows_d, to_dev_u8(new))
        for v, name in _ring_variants(qp, n):
            try:
                db.set_variant(n, v, rows=True)
            except qp.PirError:
                continue
            banner(f"incremental hint m={m} n={n} {name}")
            H.zero_()
            db.hint_update_rows(rows_d, Ad, H)
            Hh = to_host_u32(H)
            assert np.array_equal(Hh[rows], exp), name
            untouched = np.ones(R, dtype=bool)
            untouched[rows] = False
            assert not Hh[untouched].any(), name


def test_workspace_covers_every_plan(qp):
    # The reported workspace is enough for every batch size, gathered or not:
    # the calls above and these succeed with exactly that many bytes.
    import torch
    R, C = 640, 8192
    g = np.random.default_rng(5)
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    with qp.Database(to_dev_u8(D)) as db:
        for B in (1, 8, 16, 32, 33, 64, 65, 256, 1024):
            nbytes = db.workspace_bytes(B)
            ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            Q = workload.uniform_u32(g, (C, B))
            banner(f"exact workspace B={B} ({nbytes} bytes)")
            got = to_host_u32(db.answer_batch(to_dev_u32(Q), ws=ws))
            assert np.array_equal(got, oracle.answer_batch(D, Q))
            rows = workload.distinct_rows(g, R, 3)
            H = torch.zeros((R, B), dtype=torch.int32, device="cuda")
            db.hint_update_rows(to_dev_u32(rows), to_dev_u32(Q), H, ws=ws)
            assert np.array_equal(to_host_u32(H)[rows], oracle.hint(D, Q, rows=rows))


@pytest.mark.parametrize("m,n,C", [(37, 256, 16384), (300, 1024, 8192 + 48), (1, 5, 4096),
                                   (129, 64, 2064)])
def test_incremental_hint_prepared_planes(qp, m, n, C):
    """A's limb planes prepared once (pir_hint_planes), then two refreshes
    in a row whose incremental hints read them: each equals the oracle's
    hint of the refreshed rows and the call that re-derives the planes from
    A, for every variant of the gathered table (narrow ones fall back to the
    wide layout the planes use)."""
    import torch
    R = 2048
    g = np.random.default_rng(1000 + m + n)
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    A = workload.uniform_u32(g, (C, n))
    with qp.Database(to_dev_u8(D)) as db:
        Ad = to_dev_u32(A)
        planes = db.hint_planes(Ad)
        assert planes.numel() == qp.lib().pir_hint_planes_bytes(db.handle, n)
        H_pl = torch.zeros((R, n), dtype=torch.int32, device="cuda")
        H_a = torch.zeros((R, n), dtype=torch.int32, device="cuda")
        for rep in range(2):
            rows = workload.distinct_rows(g, R, m)
            new = g.integers(0, 256, size=(m, C), dtype=np.uint8)
            D = oracle.update_rows(D, rows, new)
            exp = oracle.hint(D, A, rows=rows)
            rows_d = to_dev_u32(rows)
            db.update_rows(rows_d, to_dev_u8(new))
            for v, name in [(0, "auto")] + _ring_variants(qp, n):
                try:
                    db.set_variant(n, v, rows=True)
                except qp.PirError:
                    continue
                banner(f"prepared planes m={m} n={n} C={C} rep={rep} {name}")
                db.hint_update_rows_planes(rows_d, planes, n, H_pl)
                db.hint_update_rows(rows_d, Ad, H_a)
                got = to_host_u32(H_pl)
                assert np.array_equal(got[rows], exp), name
                assert np.array_equal(got, to_host_u32(H_a)), name
        db.set_variant(n, 0, rows=True)
        # planes too small or missing: rejected, nothing written
        lib = qp.lib()
        ws = db.workspace(n)
        before = to_host_u32(H_pl)
        assert lib.pir_hint_update_rows_planes(db.handle, rows_d.data_ptr(), m, planes.data_ptr(),
                                               planes.numel() - 1, n, H_pl.data_ptr(),
                                               ws.data_ptr(), ws.numel(), None) == 6
        assert lib.pir_hint_update_rows_planes(db.handle, rows_d.data_ptr(), m, None, 0, n,
                                               H_pl.data_ptr(), ws.data_ptr(), ws.numel(),
                                               None) == 1
        torch.cuda.synchronize()
        assert np.array_equal(to_host_u32(H_pl), before)
