"""The allocation-free batched Answer (pir_answer_batch_noalloc), called
through the C ABI, against pir_answer_batch with a caller workspace: two
calls in a row, the second on a smaller input, then sizes past the fixed
scratch array rejected with nothing written."""
import ctypes

import numpy as np
import pytest

import oracle
import workload
from _util import banner, to_dev_u32, to_dev_u8, to_host_u32

pytestmark = pytest.mark.gpu
SHAPE = 2


def _batch_with_ws(lib, db, Qd, B):
    import torch
    out = torch.full((db.rows, B), -1, dtype=torch.int32, device="cuda")
    ws = db.workspace(B)
    st = lib.pir_answer_batch(db.handle, Qd.data_ptr(), B, out.data_ptr(), ws.data_ptr(),
                              ws.numel(), None)
    assert st == 0
    return out


def _batch_noalloc(lib, db, Qd, B):
    import torch
    out = torch.full((db.rows, B), -1, dtype=torch.int32, device="cuda")
    st = lib.pir_answer_batch_noalloc(db.handle, Qd.data_ptr(), B, out.data_ptr(), None)
    assert st == 0
    return out


def test_noalloc_matches_workspace_path(gpu):
    import torch
    import paper_2510_03631_amd as qp
    lib = qp.lib()
    g = workload.rng(workload.SEED_BASE + 120)
    # (rows, cols, B): the first call fills the scratch array with a larger
    # input (several tiles, a ragged tail, 2-way split-K at 64 queries); the
    # second call's smaller input must not see its leftovers.
    cases = [(4100, 8208, 64), (1000, 2064, 5), (300, 1040, 1), (3000, 4096, 33)]
    for R, C, B in cases:
        banner(f"noalloc vs workspace path: {R}x{C}, B={B}")
        D = workload.db_bytes(g, R, C)
        Q = workload.uniform_u32(g, (C, B))
        with qp.Database(to_dev_u8(D)) as db:
            Qd = to_dev_u32(Q)
            ref = to_host_u32(_batch_with_ws(lib, db, Qd, B))
            got = to_host_u32(_batch_noalloc(lib, db, Qd, B))
            torch.cuda.synchronize()
            assert np.array_equal(got, ref), (R, C, B)
            rows = np.unique(np.concatenate([[0, R - 1], g.choice(R, 40, replace=False)]))
            assert np.array_equal(got[rows], oracle.answer_batch(D[rows], Q)), (R, C, B)
            # twice in a row on the same handle: same words
            again = to_host_u32(_batch_noalloc(lib, db, Qd, B))
            assert np.array_equal(again, ref), (R, C, B)


def test_noalloc_rejects_sizes_past_the_scratch(gpu):
    import torch
    import paper_2510_03631_amd as qp
    lib = qp.lib()
    banner("noalloc: oversized batch rejected, nothing written")
    R, C = 512, 65536
    D = torch.zeros((R, C), dtype=torch.uint8, device="cuda")
    with qp.Database(D) as db:
        B = 512   # 4 * B * C bytes of limb planes = 128 MiB > the 64 MiB array
        Qd = torch.zeros((C, B), dtype=torch.int32, device="cuda")
        out = torch.full((R, B), 7, dtype=torch.int32, device="cuda")
        assert lib.pir_answer_batch_noalloc(db.handle, Qd.data_ptr(), B, out.data_ptr(),
                                            None) == SHAPE
        assert lib.pir_answer_batch_noalloc(db.handle, None, 4, out.data_ptr(), None) == 1
        assert lib.pir_answer_batch_noalloc(db.handle, Qd.data_ptr(), 0, out.data_ptr(),
                                            None) == 0
        torch.cuda.synchronize()
        assert int((out != 7).sum().item()) == 0
        # a batch that fits still runs on the same handle afterwards
        B = 8
        Q = np.random.default_rng(3).integers(0, 1 << 32, size=(C, B), dtype=np.uint32)
        Qs = to_dev_u32(Q)
        o = torch.empty((R, B), dtype=torch.int32, device="cuda")
        assert lib.pir_answer_batch_noalloc(db.handle, Qs.data_ptr(), B, o.data_ptr(), None) == 0
        torch.cuda.synchronize()
        assert int(o.abs().sum().item()) == 0   # D == 0
