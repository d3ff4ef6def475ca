"""Goldberg (FTR) field form on the GPU: ``D Q mod p`` (pir_answer_batch_modp)
against the oracle, element by element; the client round trip (Shamir
shares -> server products -> Lagrange at 0 recovers the records); the
int32 edge of an exact 2^17-column accumulation; the full 2^18-record
workload on sampled entries; error paths."""
import time

import numpy as np
import pytest

import oracle
import workload
from _util import banner, to_dev_u32, to_dev_u8, to_host_u32

pytestmark = pytest.mark.gpu
M32 = 1 << 32
P = workload.FTR_PRIME
PRIMES = (257, 65537, 2147483647, P)


@pytest.fixture(scope="module")
def qp(gpu):
    import paper_2510_03631_amd as p
    return p


@pytest.mark.parametrize("R,C,B", [(1, 16, 1), (37, 272, 3), (300, 4096, 33), (129, 1040, 64),
                                   (64, 2000, 100), (513, 512, 256), (260, 8192, 7)])
def test_modp_matches_oracle(qp, R, C, B):
    g = np.random.default_rng(R * 7 + C + B)
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    with qp.Database(to_dev_u8(D)) as db:
        for i, p in enumerate(PRIMES):
            # Residues for some cases, arbitrary words (taken as integers) for others.
            Q = workload.uniform_mod(g, (C, B), p) if i % 2 else workload.uniform_u32(g, (C, B))
            banner(f"modp R={R} C={C} B={B} p={p}")
            got = to_host_u32(db.answer_batch_modp(to_dev_u32(Q), p))
            assert np.array_equal(got, oracle.answer_batch_mod(D, Q, p)), p


def test_modp_extreme_words(qp):
    # All bytes 255 against words 2^32 - 1 and p - 1: the largest sums.
    R, C, B = 70, 4096, 40
    D = np.full((R, C), 255, dtype=np.uint8)
    Q = np.full((C, B), M32 - 1, dtype=np.uint32)
    Q[:, ::2] = P - 1
    with qp.Database(to_dev_u8(D)) as db:
        for p in PRIMES:
            banner(f"modp extremes p={p}")
            got = to_host_u32(db.answer_batch_modp(to_dev_u32(Q), p))
            assert np.array_equal(got, oracle.answer_batch_mod(D, Q, p)), p


def test_modp_every_variant(qp):
    from paper_2510_03631_amd._lib import variant_names
    R, C, B = 300, 4096, 64
    g = np.random.default_rng(11)
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    Q = workload.uniform_mod(g, (C, B), P)
    exp = oracle.answer_batch_mod(D, Q, P)
    with qp.Database(to_dev_u8(D)) as db:
        for v, name in enumerate(variant_names(B)):
            try:
                db.set_variant(B, v)
            except qp.PirError:
                continue
            # Variants without split-K serve the field form with the default
            # ring kernel; the result is the same either way.
            banner(f"modp variant {name}")
            assert np.array_equal(to_host_u32(db.answer_batch_modp(to_dev_u32(Q), P)), exp), name


@pytest.mark.parametrize("R,C,B", [(300, 4096, 3), (517, 8192, 8), (64, 2048, 16),
                                   (40, (1 << 17) + 4096, 8)])
def test_modp_small_batch_variants(qp, R, C, B):
    # Every variant that serves a small batch (dot4 stream, narrow and wide
    # matrix-core layouts, split-K when C > 2^17) gives the oracle's value.
    from paper_2510_03631_amd._lib import variant_names
    g = np.random.default_rng(R + C + B)
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    Q = workload.uniform_mod(g, (C, B), P)
    exp = oracle.answer_batch_mod(D, Q, P)
    tried = 0
    with qp.Database(to_dev_u8(D)) as db:
        for v, name in enumerate(variant_names(B)):
            if not name.startswith(("ring", "narrow", "few")):
                continue
            try:
                db.set_variant(B, v)
            except qp.PirError:
                continue
            banner(f"modp small batch R={R} C={C} B={B} {name}")
            assert np.array_equal(to_host_u32(db.answer_batch_modp(to_dev_u32(Q), P)), exp), name
            tried += 1
    assert tried >= 3


def test_modp_rows_longer_than_one_exact_span(qp):
    # C > 2^17: every accumulation covers at most 2^17 columns (split-K).
    R, C, B = 40, (1 << 17) + 4096, 5
    g = np.random.default_rng(12)
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    Q = workload.uniform_u32(g, (C, B))
    banner(f"modp long rows R={R} C={C} B={B}")
    with qp.Database(to_dev_u8(D)) as db:
        got = to_host_u32(db.answer_batch_modp(to_dev_u32(Q), P))
    assert np.array_equal(got, oracle.answer_batch_mod(D, Q, P))


def test_modp_full_span_int32_edge(qp):
    """One accumulation over exactly 2^17 columns of centred bytes -128 x -128
    sums to +2^31, which an int32 accumulator reads as -2^31.

    Zero database rows against query words whose low byte (or every byte) is
    zero produce exactly that limb product; their answers must be 0.  The
    shape (8192 rows, 1024 queries, 256 x 256 tiles: 512 tiles, two per CU)
    needs no split for occupancy, so each accumulation spans all 2^17
    columns."""
    import torch
    R, C, B = 8192, 1 << 17, 1024
    t0 = time.perf_counter()
    banner(f"modp int32 edge R={R} C={C} B={B}")
    D = workload.device_db(R, C, workload.SEED_BASE + 31, "cuda")
    D[: R // 2].zero_()
    Q = workload.device_mod((C, B), P, workload.SEED_BASE + 32, "cuda")
    Q &= ~0xFF                                        # low byte zero everywhere
    Q[:, :8] = 0                                      # every byte zero
    with qp.Database(D) as db:
        db.set_variant(B, "ring8w_256x256_k128_s2")
        out = db.answer_batch_modp(Q, P)
        torch.cuda.synchronize()
    print(f"  [{time.perf_counter() - t0:6.1f}s] product done", flush=True)
    assert int(out[: R // 2].abs().max()) == 0
    g = np.random.default_rng(13)
    rs = g.integers(R // 2, R, size=48)
    bs = g.integers(0, B, size=48)
    rs[:4], bs[:4] = R - 1, [0, 7, 8, B - 1]
    Dr = D[torch.from_numpy(rs).cuda()].cpu().numpy()
    Qc = Q[:, torch.from_numpy(bs).cuda()].t().contiguous().cpu().numpy().view(np.uint32)
    exp = oracle.answer_mod_entries(Dr, Qc, P)
    got = to_host_u32(out[torch.from_numpy(rs).cuda(), torch.from_numpy(bs).cuda()])
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("servers,t", [(4, 2), (3, 1)])
def test_goldberg_round_trip(qp, servers, t):
    """Client shares (oracle) -> server products (GPU) -> interpolation
    (oracle) recovers the retrieved records from any t + 1 servers."""
    R, C = workload.FTR_RECORD_BYTES, 4096            # 4096 records of 3 KB
    g = np.random.default_rng(servers * 31 + t)
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    thetas = [int(x) for x in g.choice(C, size=8, replace=False)]
    alphas = list(range(1, servers + 1))
    Qs = np.zeros((servers, C, len(thetas)), dtype=np.uint32)
    for b, th in enumerate(thetas):
        e = np.zeros(C, dtype=np.uint32)
        e[th] = 1
        Qs[:, :, b] = oracle.shamir_shares(e, workload.uniform_mod(g, (t, C), P), alphas, P)
    resp = []
    with qp.Database(to_dev_u8(D)) as db:
        for i in range(servers):
            banner(f"goldberg server {i} of {servers} (t={t})")
            resp.append(to_host_u32(db.answer_batch_modp(to_dev_u32(Qs[i]), P)))
    assert np.array_equal(resp[0], oracle.answer_batch_mod(D, Qs[0], P))
    want = D[:, thetas].astype(np.uint32)
    for pick in (list(range(t + 1)), list(range(servers - t - 1, servers))):
        got = oracle.lagrange_at_zero([alphas[i] for i in pick], [resp[i] for i in pick], P)
        assert np.array_equal(got, want)


@pytest.mark.parametrize("B", workload.FTR_BATCHES)
def test_ftr_fullsize_sampled(qp, B):
    """The 2^18-record database (3072 x 262144 bytes, 768 MiB) with share
    batches of 1, 128 and 1024: sampled entries against the oracle."""
    import torch
    R, C = workload.FTR_RECORD_BYTES, workload.FTR_RECORDS[-1]
    banner(f"ftr full size R={R} C={C} B={B}")
    D = workload.device_db(R, C, workload.SEED_BASE + 41, "cuda")
    Q = workload.device_mod((C, B), P, workload.SEED_BASE + 42 + B, "cuda")
    with qp.Database(D) as db:
        out = db.answer_batch_modp(Q, P)
        torch.cuda.synchronize()
    g = np.random.default_rng(B)
    k = 64
    rs = g.integers(0, R, size=k)
    bs = g.integers(0, B, size=k)
    rs[0], bs[0] = R - 1, B - 1
    rt, bt = torch.from_numpy(rs).cuda(), torch.from_numpy(bs).cuda()
    exp = oracle.answer_mod_entries(D[rt].cpu().numpy(),
                                    Q[:, bt].t().contiguous().cpu().numpy().view(np.uint32), P)
    assert np.array_equal(to_host_u32(out[rt, bt]), exp)
    assert int((out.to(torch.int64) & 0xFFFFFFFF).max()) < P


def test_modp_error_paths(qp):
    import torch
    from paper_2510_03631_amd._lib import lib
    INVALID_ARG, SHAPE, UNSUPPORTED = 1, 2, 5
    banner("modp error paths")
    D = torch.zeros((64, 128), dtype=torch.uint8, device="cuda")
    Q = torch.zeros((128, 4), dtype=torch.int32, device="cuda")
    out = torch.zeros((64, 4), dtype=torch.int32, device="cuda")
    with qp.Database(D) as db:
        ws = db.workspace(4)
        for p in (0, 1):
            st = lib().pir_answer_batch_modp(db.handle, Q.data_ptr(), 4, p, out.data_ptr(),
                                             ws.data_ptr(), ws.numel(), None)
            assert st == INVALID_ARG
        with pytest.raises(ValueError):
            db.answer_batch_modp(Q, 1)
        # B == 0 is a no-op; a missing workspace is rejected.
        assert lib().pir_answer_batch_modp(db.handle, Q.data_ptr(), 0, P, out.data_ptr(),
                                           None, 0, None) == 0
        assert lib().pir_answer_batch_modp(db.handle, Q.data_ptr(), 4, P, out.data_ptr(),
                                           None, 0, None) == 6
        torch.cuda.synchronize()
    # Unaligned rows: beyond 4 queries the field form needs the ring kernels.
    store = torch.zeros(64 * 128 + 1, dtype=torch.uint8, device="cuda")
    Q5 = torch.zeros((128, 5), dtype=torch.int32, device="cuda")
    with qp.Database(store[1:].view(64, 128)) as db:
        with pytest.raises(qp.PirError) as ei:
            db.answer_batch_modp(Q5, P)
        assert ei.value.status == UNSUPPORTED
    # More than 2^23 columns (checked before the workspace).
    wide = torch.zeros((1, (1 << 23) + 16), dtype=torch.uint8, device="cuda")
    Qw = torch.zeros(((1 << 23) + 16, 1), dtype=torch.int32, device="cuda")
    o1 = torch.zeros((1, 1), dtype=torch.int32, device="cuda")
    with qp.Database(wide) as db:
        assert lib().pir_answer_batch_modp(db.handle, Qw.data_ptr(), 1, P, o1.data_ptr(),
                                           None, 0, None) == SHAPE
    torch.cuda.synchronize()
    assert out.abs().max().item() == 0 and o1.abs().max().item() == 0   # nothing written
