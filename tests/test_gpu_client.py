"""Client-side LWE steps on the GPU against the oracle's client, and the
full round trip query -> answer -> decode on the device."""
import numpy as np
import pytest

import oracle
import workload
from _util import banner, to_dev_u32, to_dev_u8, to_host_u32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qp(gpu):
    import paper_2510_03631_amd as p
    return p


def _dev_i32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to("cuda")


@pytest.mark.parametrize("R,C,n,B", [(1024, 1024, 1024, 3), (333, 1000, 77, 17),
                                     (64, 2048, 1500, 1), (2000, 300, 64, 40),
                                     (100, 512, 1030, 5), (1001, 1023, 256, 9)])
def test_client_query_decode_round_trip(qp, R, C, n, B):
    banner(f"client round trip R={R} C={C} n={n} B={B}")
    g = workload.rng(R + C + n + B)
    D = workload.db_bytes(g, R, C)
    A = workload.uniform_u32(g, (C, n))
    dr = workload.lwe_draws(g, C, n, B)
    Ad = to_dev_u32(A)
    Qt = qp.client_query(Ad, to_dev_u32(dr.s), _dev_i32(dr.e), to_dev_u32(dr.col.astype(np.uint32)))
    Qt_h = to_host_u32(Qt)
    for b in range(B):
        assert np.array_equal(Qt_h[b], oracle.lwe_query(A, dr.s[b], dr.e[b], int(dr.col[b]))), b
    with qp.Database(to_dev_u8(D)) as db:
        H = db.setup_hint(Ad)
        ans = db.answer_batch_qmajor(Qt) if B > 1 else db.answer(Qt[0]).view(1, R)
        m = qp.client_decode(H, to_dev_u32(dr.s), ans).cpu().numpy()
        H_h = to_host_u32(H)
        ans_h = to_host_u32(ans)
    for b in range(B):
        assert np.array_equal(m[b], oracle.lwe_decode(ans_h[b], H_h, dr.s[b])), b
        assert np.array_equal(m[b], D[:, int(dr.col[b])]), b


def test_client_unaligned_matrix(qp):
    """A public matrix that starts 4 bytes into its allocation takes the
    word-load path (n % 4 == 0 but not 16-byte aligned); same results."""
    import torch
    banner("client query, unaligned matrix")
    g = workload.rng(31337)
    C, n, B = 700, 512, 3
    A = workload.uniform_u32(g, (C, n))
    dr = workload.lwe_draws(g, C, n, B)
    store = torch.zeros(C * n + 1, dtype=torch.int32, device="cuda")
    store[1:] = to_dev_u32(A).view(-1)
    Ad = store[1:].view(C, n)
    assert Ad.data_ptr() % 16 != 0
    Qt = to_host_u32(qp.client_query(Ad, to_dev_u32(dr.s), _dev_i32(dr.e),
                                     to_dev_u32(dr.col.astype(np.uint32))))
    for b in range(B):
        assert np.array_equal(Qt[b], oracle.lwe_query(A, dr.s[b], dr.e[b], int(dr.col[b]))), b


def test_client_decode_boundaries(qp):
    """Noise at the rounding edges, with H = 0 so the answer is m * 2^24 + noise."""
    import torch
    banner("client decode rounding boundaries")
    m = np.array([0, 7, 255, 0, 100, 255], dtype=np.int64)
    noise = np.array([(1 << 23) - 1, -(1 << 23), 0, -1, 1 << 23, (1 << 23) - 1])
    a = (((m << 24) + noise) % (1 << 32)).astype(np.uint32).reshape(1, 6)
    H = torch.zeros((6, 5), dtype=torch.int32, device="cuda")
    S = torch.zeros((1, 5), dtype=torch.int32, device="cuda")
    out = qp.client_decode(H, S, to_dev_u32(a)).cpu().numpy()[0]
    assert out.tolist() == oracle.lwe_decode(a[0], np.zeros((6, 5), np.uint32),
                                             np.zeros(5, np.uint32)).tolist()
    assert out.tolist() == [0, 7, 255, 0, 101, 255]


def test_client_full_size(qp):
    """32768 x 1024 public matrix, 4 queries, against the oracle."""
    banner("client query 32768x1024, B=4")
    g = workload.rng(workload.SEED_BASE + 1)
    C, n, B = 32768, 1024, 4
    A = workload.uniform_u32(g, (C, n))
    dr = workload.lwe_draws(g, C, n, B)
    Qt = to_host_u32(qp.client_query(to_dev_u32(A), to_dev_u32(dr.s), _dev_i32(dr.e),
                                     to_dev_u32(dr.col.astype(np.uint32))))
    for b in range(B):
        assert np.array_equal(Qt[b], oracle.lwe_query(A, dr.s[b], dr.e[b], int(dr.col[b])))


def test_client_errors(qp):
    banner("client argument errors")
    lib = qp.lib()
    assert lib.pir_client_query(None, 4, 4, None, None, None, 1, None, None) == 1
    import torch
    t = torch.zeros(16, dtype=torch.int32, device="cuda")
    p = t.data_ptr()
    assert lib.pir_client_query(p, 0, 4, p, p, p, 1, p, None) == 2
    assert lib.pir_client_decode(p, 4, 4, p, p, 0, p, None) == 2


@pytest.mark.parametrize("R,C,n,B", [(1024, 1024, 1024, 16), (333, 1000, 77, 17),
                                     (2000, 300, 64, 40), (100, 512, 1030, 5),
                                     (1001, 1023, 256, 64), (64, 2048, 12, 1)])
def test_client_matrix_core_round_trip(qp, R, C, n, B):
    """The matrix-core client steps (A and H as byte planes under the
    batched Answer) against the oracle's client: every query word, every
    decoded byte, and the word path's outputs bit for bit.  n = 77 and 1030
    give 4n not a multiple of 16 (the register-staged kernels); a ragged
    batch of 17 and 40 pads the limb layout."""
    banner(f"client matrix cores R={R} C={C} n={n} B={B}")
    g = workload.rng(7 * R + C + n + B)
    D = workload.db_bytes(g, R, C)
    A = workload.uniform_u32(g, (C, n))
    dr = workload.lwe_draws(g, C, n, B)
    Ad, Sd = to_dev_u32(A), to_dev_u32(dr.s)
    Ed, cd = _dev_i32(dr.e), to_dev_u32(dr.col.astype(np.uint32))
    with qp.ClientMatrix(Ad) as Am:
        Qt = Am.query(Sd, Ed, cd)
        Qt_h = to_host_u32(Qt)
        for b in range(B):
            assert np.array_equal(Qt_h[b], oracle.lwe_query(A, dr.s[b], dr.e[b], int(dr.col[b]))), b
        assert np.array_equal(Qt_h, to_host_u32(qp.client_query(Ad, Sd, Ed, cd)))
        Qt2 = to_host_u32(Am.query(Sd, Ed, cd))          # the same handle again
        assert np.array_equal(Qt2, Qt_h)
    with qp.Database(to_dev_u8(D)) as db:
        H = db.setup_hint(Ad)
        ans = db.answer_batch_qmajor(Qt) if B > 1 else db.answer(Qt[0]).view(1, R)
    H_h, ans_h = to_host_u32(H), to_host_u32(ans)
    with qp.ClientMatrix(H) as Hm:
        m = Hm.decode(Sd, ans).cpu().numpy()
    for b in range(B):
        assert np.array_equal(m[b], oracle.lwe_decode(ans_h[b], H_h, dr.s[b])), b
        assert np.array_equal(m[b], D[:, int(dr.col[b])]), b


def test_client_matrix_core_full_size(qp):
    """32768 x 1024 public matrix and hint-shaped matrix, 64 secrets: every
    query word against the oracle; decode against the oracle's decode of
    uniform answers (a decode is defined for any answer words)."""
    banner("client matrix cores 32768x1024, B=64")
    g = workload.rng(workload.SEED_BASE + 2)
    C, n, B = 32768, 1024, 64
    A = workload.uniform_u32(g, (C, n))
    dr = workload.lwe_draws(g, C, n, B)
    Sd = to_dev_u32(dr.s)
    with qp.ClientMatrix(to_dev_u32(A)) as Am:
        Qt = to_host_u32(Am.query(Sd, _dev_i32(dr.e), to_dev_u32(dr.col.astype(np.uint32))))
    for b in range(0, B, 7):
        assert np.array_equal(Qt[b], oracle.lwe_query(A, dr.s[b], dr.e[b], int(dr.col[b]))), b
    ans = workload.uniform_u32(g, (B, C))
    with qp.ClientMatrix(to_dev_u32(A)) as Hm:
        m = Hm.decode(Sd, to_dev_u32(ans)).cpu().numpy()
    for b in range(0, B, 9):
        assert np.array_equal(m[b], oracle.lwe_decode(ans[b], A, dr.s[b])), b


def test_client_matrix_core_errors(qp):
    import torch
    banner("client matrix cores: argument errors")
    import ctypes
    lib = qp.lib()
    out = ctypes.c_void_p()
    assert lib.pir_client_mat_open(None, 4, 4, None, ctypes.byref(out)) == 1
    t = torch.zeros(64, dtype=torch.int32, device="cuda")
    assert lib.pir_client_mat_open(t.data_ptr(), 0, 4, None, ctypes.byref(out)) == 2
    assert lib.pir_client_mat_workspace_bytes(None, 4) == 0
    with qp.ClientMatrix(t.view(16, 4)) as m:
        S = torch.zeros((2, 4), dtype=torch.int32, device="cuda")
        E = torch.zeros((2, 16), dtype=torch.int32, device="cuda")
        cols = torch.zeros(2, dtype=torch.int32, device="cuda")
        Qt = torch.full((2, 16), 5, dtype=torch.int32, device="cuda")
        ws = m.workspace(2)
        assert lib.pir_client_query_mat(m._h, S.data_ptr(), E.data_ptr(), cols.data_ptr(), 2,
                                        Qt.data_ptr(), ws.data_ptr(), ws.numel() - 1, None) == 6
        assert lib.pir_client_query_mat(m._h, S.data_ptr(), E.data_ptr(), cols.data_ptr(), 0,
                                        Qt.data_ptr(), ws.data_ptr(), ws.numel(), None) == 2
        torch.cuda.synchronize()
        assert int((Qt != 5).sum().item()) == 0   # nothing written


def test_client_matrix_core_every_variant(qp):
    """Every product variant a prepared client matrix can take gives the
    oracle's queries (the secrets' operand is written straight into the
    wide limb layout, which every wide variant reads)."""
    from paper_2510_03631_amd._lib import variant_names
    banner("client matrix cores: every variant")
    g = workload.rng(4711)
    C, n, B = 700, 128, 40
    A = workload.uniform_u32(g, (C, n))
    dr = workload.lwe_draws(g, C, n, B)
    exp = np.stack([oracle.lwe_query(A, dr.s[b], dr.e[b], int(dr.col[b])) for b in range(B)])
    tried = 0
    with qp.ClientMatrix(to_dev_u32(A)) as Am:
        Sd, Ed = to_dev_u32(dr.s), _dev_i32(dr.e)
        cd = to_dev_u32(dr.col.astype(np.uint32))
        for v, name in enumerate(variant_names(B)):
            try:
                Am.set_variant(B, v)
            except qp.PirError:
                continue
            banner(f"client matrix cores variant {name}")
            assert np.array_equal(to_host_u32(Am.query(Sd, Ed, cd)), exp), name
            tried += 1
    assert tried >= 4
