"""GPU parity: the HIP path against the CPU oracle, element by element.

Integers throughout, so the bar is bit-exact equality.  Sizes here finish in
seconds on the oracle while spanning several tiles and ragged tails; the
gigabyte configurations are in test_gpu_fullsize.py.
"""
import numpy as np
import pytest

import oracle
import workload
from _util import banner, lwe_queries, to_dev_u32, to_dev_u8, to_host_u32

pytestmark = pytest.mark.gpu
M32 = 1 << 32


@pytest.fixture(scope="module")
def qp(gpu):
    import paper_2510_03631_amd as p
    return p


def _db(qp, D_host, pitch_pad=0, offset=0):
    """Open a database on a copy of D_host, optionally with padded rows or an
    odd base address (exercises the unaligned kernels)."""
    import torch
    R, C = D_host.shape
    if pitch_pad or offset:
        store = torch.zeros(R * (C + pitch_pad) + offset + 16, dtype=torch.uint8, device="cuda")
        view = store[offset:offset + R * (C + pitch_pad)].view(R, C + pitch_pad)[:, :C]
        view.copy_(to_dev_u8(D_host))
        return qp.Database(view), view
    Dd = to_dev_u8(D_host)
    return qp.Database(Dd), Dd


# ------------------------------------------------------------------ tiny LWE
def test_tiny_lwe_answer_hint_decode(qp):
    """1024 x 1024 database, n = 1024: answer and hint bit-exact, and the
    client decodes the queried column from the GPU's outputs."""
    import torch
    banner("tiny 1024x1024 LWE answer + hint")
    g = workload.rng(workload.SEED_BASE)
    R = C = n = 1024
    D = workload.db_bytes(g, R, C)
    A = workload.uniform_u32(g, (C, n))
    dr = workload.lwe_draws(g, C, n, 1)
    q = oracle.lwe_query(A, dr.s[0], dr.e[0], int(dr.col[0]))
    db, _ = _db(qp, D)
    a = to_host_u32(db.answer(to_dev_u32(q)))
    H = to_host_u32(db.setup_hint(to_dev_u32(A)))
    torch.cuda.synchronize()
    assert np.array_equal(a, oracle.answer(D, q))
    assert np.array_equal(H, oracle.hint(D, A))
    assert np.array_equal(oracle.lwe_decode(a, H, dr.s[0]), D[:, int(dr.col[0])])
    db.close()


# ------------------------------------------------------------------ single query, ragged
SHAPES = [(1, 1), (1, 17), (3, 1000), (64, 1024), (65, 1025), (100, 4097), (257, 5000),
          (1000, 3), (129, 8191), (37, 12289)]


@pytest.mark.parametrize("R,C", SHAPES)
@pytest.mark.parametrize("layout", ["aligned", "pitch+3", "offset+1"])
def test_answer_ragged(qp, R, C, layout):
    banner(f"answer R={R} C={C} layout={layout}")
    g = np.random.default_rng(R * 7919 + C)
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    q = g.integers(0, M32, size=C, dtype=np.uint32)
    if layout == "aligned":
        db, _ = _db(qp, D)
    elif layout == "pitch+3":
        db, _ = _db(qp, D, pitch_pad=3)
    else:
        db, _ = _db(qp, D, offset=1)
    got = to_host_u32(db.answer(to_dev_u32(q)))
    assert np.array_equal(got, oracle.answer(D, q))
    db.close()


def test_answer_unaligned_query(qp):
    import torch
    banner("answer with a query at an odd word offset")
    g = np.random.default_rng(5)
    R, C = 70, 3000
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    q = g.integers(0, M32, size=C, dtype=np.uint32)
    db, _ = _db(qp, D)
    buf = torch.zeros(C + 1, dtype=torch.int32, device="cuda")
    buf[1:].copy_(to_dev_u32(q))
    got = to_host_u32(db.answer(buf[1:]))
    assert np.array_equal(got, oracle.answer(D, q))
    db.close()


@pytest.mark.parametrize("R,C", [(64, 50000), (1, 70000), (300, 9000), (4096, 4096)])
def test_answer_split_columns(qp, R, C):
    """Few row blocks: the column range is split and partial sums are added."""
    banner(f"answer split R={R} C={C}")
    g = np.random.default_rng(R + C)
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    q = g.integers(0, M32, size=C, dtype=np.uint32)
    db, _ = _db(qp, D)
    got = to_host_u32(db.answer(to_dev_u32(q)))
    assert np.array_equal(got, oracle.answer(D, q))
    db.close()


def test_answer_extremes(qp):
    banner("answer extreme values")
    R, C = 65, 2049
    for dval, qval in [(0, 0), (255, 0xFFFFFFFF), (0x80, 0x80808080), (255, 0xFF)]:
        D = np.full((R, C), dval, dtype=np.uint8)
        q = np.full(C, qval, dtype=np.uint32)
        db, _ = _db(qp, D)
        got = to_host_u32(db.answer(to_dev_u32(q)))
        assert np.array_equal(got, oracle.answer(D, q)), (dval, qval)
        db.close()


# ------------------------------------------------------------------ batch
BATCH_SHAPES = [(1, 1), (5, 33), (130, 1000), (257, 4097), (64, 256), (300, 777)]


@pytest.mark.parametrize("R,C", BATCH_SHAPES)
@pytest.mark.parametrize("B", [1, 2, 3, 31, 32, 33, 64, 65, 130])
def test_batch_ragged(qp, R, C, B):
    banner(f"batch R={R} C={C} B={B}")
    g = np.random.default_rng(R * 131 + C * 7 + B)
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    Q = g.integers(0, M32, size=(C, B), dtype=np.uint32)
    db, _ = _db(qp, D)
    got = to_host_u32(db.answer_batch(to_dev_u32(Q)))
    assert np.array_equal(got, oracle.answer_batch(D, Q))
    db.close()


@pytest.mark.parametrize("layout", ["pitch+3", "offset+1"])
def test_batch_unaligned(qp, layout):
    banner(f"batch unaligned {layout}")
    g = np.random.default_rng(17)
    R, C, B = 150, 1500, 40
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    Q = g.integers(0, M32, size=(C, B), dtype=np.uint32)
    db, _ = _db(qp, D, pitch_pad=3) if layout == "pitch+3" else _db(qp, D, offset=1)
    got = to_host_u32(db.answer_batch(to_dev_u32(Q)))
    assert np.array_equal(got, oracle.answer_batch(D, Q))
    db.close()


def test_batch_column_equals_single(qp):
    banner("batch column == single answer")
    g = np.random.default_rng(23)
    R, C, B = 513, 3000, 64
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    Q = g.integers(0, M32, size=(C, B), dtype=np.uint32)
    db, _ = _db(qp, D)
    out = to_host_u32(db.answer_batch(to_dev_u32(Q)))
    for b in (0, 17, 63):
        single = to_host_u32(db.answer(to_dev_u32(np.ascontiguousarray(Q[:, b]))))
        assert np.array_equal(out[:, b], single)
    db.close()


def test_batch_extremes_and_wrap(qp):
    """Centred products (-128)(-128) summed over C = 131072 reach 2^31 and
    wrap the int32 accumulator; the answers must still be exact."""
    banner("batch accumulator wrap C=131072")
    R, C, B = 64, 131072, 8
    for dval, qval in [(0, 0), (255, 0xFFFFFFFF), (0, 0x80808080), (255, 0x7F7F7F7F)]:
        D = np.full((R, C), dval, dtype=np.uint8)
        Q = np.full((C, B), qval, dtype=np.uint32)
        db, _ = _db(qp, D)
        got = to_host_u32(db.answer_batch(to_dev_u32(Q)))
        exp = (dval * qval * C) % M32
        assert (got == exp).all(), (dval, qval)
        assert np.array_equal(got, oracle.answer_batch(D, Q))
        db.close()


def test_single_wrap(qp):
    banner("answer wrap C=131072")
    R, C = 64, 131072
    g = np.random.default_rng(2)
    D = np.zeros((R, C), dtype=np.uint8)
    D[1::2] = 255
    q = g.integers(0, M32, size=C, dtype=np.uint32)
    db, _ = _db(qp, D)
    got = to_host_u32(db.answer(to_dev_u32(q)))
    assert np.array_equal(got, oracle.answer(D, q))
    db.close()


# ------------------------------------------------------------------ hint + update
@pytest.mark.parametrize("R,C,n", [(300, 777, 64), (1000, 1024, 256), (77, 5000, 33)])
def test_hint_and_incremental_update(qp, R, C, n):
    import torch
    banner(f"hint + row update R={R} C={C} n={n}")
    g = np.random.default_rng(R + C + n)
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    A = g.integers(0, M32, size=(C, n), dtype=np.uint32)
    db, Dd = _db(qp, D)
    Ad = to_dev_u32(A)
    Hd = db.setup_hint(Ad)
    assert np.array_equal(to_host_u32(Hd), oracle.hint(D, A))
    m = max(1, workload.update_count(R, 0.03))
    rows = workload.distinct_rows(g, R, m)
    new = g.integers(0, 256, size=(m, C), dtype=np.uint8)
    rows_d = to_dev_u32(rows)
    db.update_rows(rows_d, to_dev_u8(new))
    db.hint_update_rows(rows_d, Ad, Hd)
    torch.cuda.synchronize()
    D2 = oracle.update_rows(D, rows, new)
    assert np.array_equal(Dd.cpu().numpy(), D2)
    assert np.array_equal(to_host_u32(Hd), oracle.hint(D2, A))
    # answers after the refresh see the new rows (metadata refreshed too)
    Q = g.integers(0, M32, size=(C, 40), dtype=np.uint32)
    assert np.array_equal(to_host_u32(db.answer_batch(to_dev_u32(Q))), oracle.answer_batch(D2, Q))
    q = Q[:, 0].copy()
    assert np.array_equal(to_host_u32(db.answer(to_dev_u32(q))), oracle.answer(D2, q))
    db.close()


def test_update_rows_unaligned_width(qp):
    import torch
    banner("row update, width not a multiple of 16")
    g = np.random.default_rng(44)
    R, C = 50, 1001
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    db, Dd = _db(qp, D)
    rows = np.array([0, 7, 49], dtype=np.uint32)
    new = g.integers(0, 256, size=(3, C), dtype=np.uint8)
    db.update_rows(to_dev_u32(rows), to_dev_u8(new))
    torch.cuda.synchronize()
    D2 = oracle.update_rows(D, rows, new)
    assert np.array_equal(Dd.cpu().numpy(), D2)
    Q = g.integers(0, M32, size=(C, 5), dtype=np.uint32)
    assert np.array_equal(to_host_u32(db.answer_batch(to_dev_u32(Q))), oracle.answer_batch(D2, Q))
    db.close()


# ------------------------------------------------------------------ determinism + errors
def test_repeat_bit_identical(qp):
    banner("repeat determinism")
    g = np.random.default_rng(8)
    R, C, B = 700, 3333, 70
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    Q = to_dev_u32(g.integers(0, M32, size=(C, B), dtype=np.uint32))
    db, _ = _db(qp, D)
    first = to_host_u32(db.answer_batch(Q))
    for _ in range(3):
        assert np.array_equal(to_host_u32(db.answer_batch(Q)), first)
    db.close()


def test_error_paths(qp):
    import torch
    banner("error paths")
    D = torch.zeros((16, 64), dtype=torch.uint8, device="cuda")
    db = qp.Database(D)
    lib = qp.lib()
    q = torch.zeros(64, dtype=torch.int32, device="cuda")
    a = torch.zeros(16, dtype=torch.int32, device="cuda")
    Q = torch.zeros((64, 4), dtype=torch.int32, device="cuda")
    out = torch.zeros((16, 4), dtype=torch.int32, device="cuda")
    h = db.handle
    assert lib.pir_answer(h, None, a.data_ptr(), None, 0, None) == 1
    assert lib.pir_answer_batch(h, Q.data_ptr(), 0, out.data_ptr(), None, 0, None) == 0
    ws_need = db.workspace_bytes(4)
    assert ws_need > 0
    ws = torch.empty(ws_need, dtype=torch.uint8, device="cuda")
    assert lib.pir_answer_batch(h, Q.data_ptr(), 4, out.data_ptr(), None, 0, None) == 6
    assert lib.pir_answer_batch(h, Q.data_ptr(), 4, out.data_ptr(), ws.data_ptr(), ws_need - 1, None) == 6
    assert lib.pir_answer_batch(h, Q.data_ptr(), 4, out.data_ptr(), ws.data_ptr() + 4, ws_need, None) == 6
    out.fill_(7)
    torch.cuda.synchronize()
    assert (out == 7).all()   # untouched after the rejected calls
    assert lib.pir_setup_hint(h, Q.data_ptr(), 0, out.data_ptr(), None, 0, None) == 1
    db.close()
    with pytest.raises(qp.PirError):
        db.answer(q)
