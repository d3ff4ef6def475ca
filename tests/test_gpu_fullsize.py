"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times.

The oracle cannot recompute gigabyte products in test time, so each case
checks (a) sampled rows element by element against the oracle, (b) the LWE
decode of every row, which recovers the queried column only if every answer
word is right to within the noise margin (and the sampled rows pin it
exactly), and (c) Freivalds' randomized check of every whole product over
all rows, 16 trials each: a wrong word anywhere survives a trial with
probability at most 1/2, so all 16 with at most 2^-16.  Databases are drawn
on the device with a seeded torch generator and copied back to the host
whole for the checks.
"""
import time

import numpy as np
import pytest

import oracle
import workload
from _util import banner, lwe_queries, sample_rows, to_dev_u32, to_dev_u8, to_host_u32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qp(gpu):
    import paper_2510_03631_amd as p
    return p


@pytest.fixture(scope="module")
def tune(qp):
    from paper_2510_03631_amd import tune as t
    return t


def _step(msg, t0):
    print(f"  [{time.perf_counter() - t0:7.1f}s] {msg}", flush=True)


@pytest.fixture(scope="module")
def spectrum(qp, tune):
    """The 32768 x 32768 database with its public matrix A (n = 1024)."""
    import torch
    t0 = time.perf_counter()
    banner("spectrum 32768x32768 setup")
    shape = workload.CONFIGS["spectrum_1q"]
    R, C, n = shape.rows, shape.cols, shape.n
    D = workload.device_db(R, C, workload.SEED_BASE + 1, "cuda")
    Dh = D.cpu().numpy()
    g = workload.rng(workload.SEED_BASE + 1)
    A = workload.uniform_u32(g, (C, n))
    Ad = to_dev_u32(A)
    db = qp.Database(D)
    tune.apply(db)   # the variants the benchmark runs
    H = db.setup_hint(Ad)
    torch.cuda.synchronize()
    _step("database, A and hint ready", t0)
    yield dict(D=D, Dh=Dh, A=A, Ad=Ad, db=db, H=H, g=g, R=R, C=C, n=n)
    db.close()
    del D, Ad, H
    torch.cuda.empty_cache()


def test_spectrum_hint(spectrum):
    t0 = time.perf_counter()
    banner("spectrum hint: sampled rows + 16 Freivalds trials over all rows")
    s = spectrum
    H = to_host_u32(s["H"])
    rows = sample_rows(s["R"], 48, 1)
    assert np.array_equal(H[rows], oracle.hint(s["Dh"][rows], s["A"]))
    _step("sampled hint rows exact", t0)
    assert oracle.freivalds(s["Dh"], s["A"], H, trials=16, seed=3)
    _step("Freivalds, 16 trials, all rows", t0)


def test_spectrum_single_query(spectrum):
    t0 = time.perf_counter()
    banner("spectrum_1q: one LWE query, 32768x32768")
    s = spectrum
    dr = workload.lwe_draws(s["g"], s["C"], s["n"], 4)
    Q = lwe_queries(s["A"], dr)
    H = to_host_u32(s["H"])
    for b in range(4):
        q = np.ascontiguousarray(Q[:, b])
        a = to_host_u32(s["db"].answer(to_dev_u32(q)))
        rows = sample_rows(s["R"], 256, 10 + b)
        assert np.array_equal(a[rows], oracle.answer(s["D"][rows].cpu().numpy(), q))
        col = int(dr.col[b])
        assert np.array_equal(oracle.lwe_decode(a, H, dr.s[b]), s["D"][:, col].cpu().numpy())
        _step(f"query {b}: sampled rows exact, all rows decode", t0)
    # a uniform query word vector as well
    q = workload.uniform_u32(s["g"], s["C"])
    a = to_host_u32(s["db"].answer(to_dev_u32(q)))
    slab = s["D"][:4096].cpu().numpy()
    assert np.array_equal(a[:4096], oracle.answer(slab, q))
    _step("uniform query: rows 0..4095 exact", t0)


def test_spectrum_batch64(spectrum):
    t0 = time.perf_counter()
    banner("spectrum_b64: 64 LWE queries, 32768x32768")
    s = spectrum
    dr = workload.lwe_draws(s["g"], s["C"], s["n"], 64)
    Q = lwe_queries(s["A"], dr)
    _step("64 queries built", t0)
    Qd = to_dev_u32(Q)
    out = to_host_u32(s["db"].answer_batch(Qd))
    rows = sample_rows(s["R"], 128, 21)
    assert np.array_equal(out[rows], oracle.answer_batch(s["Dh"][rows], Q))
    _step("sampled rows exact", t0)
    H = to_host_u32(s["H"])
    for b in range(64):
        col = int(dr.col[b])
        assert np.array_equal(oracle.lwe_decode(out[:, b], H, dr.s[b]),
                              s["D"][:, col].cpu().numpy()), b
    _step("all 64 queries decode on every row", t0)
    assert oracle.freivalds(s["Dh"], Q, out, trials=16, seed=5)
    for b in (0, 63):
        single = to_host_u32(s["db"].answer(to_dev_u32(np.ascontiguousarray(Q[:, b]))))
        assert np.array_equal(single, out[:, b])
    _step("Freivalds (16 trials, all rows) + batch column == single answer", t0)


def test_large_batch256_update(qp, tune):
    """131072 x 131072 (16 GiB) database, 256 queries and the hint; then 1% of
    the rows (1311) are rewritten and the hint is updated for those rows."""
    import torch
    t0 = time.perf_counter()
    banner("large_b256: 131072x131072, B=256, hint, 1311-row update")
    shape = workload.CONFIGS["large_b256"]
    R, C, n, B = shape.rows, shape.cols, shape.n, shape.batch
    D = workload.device_db(R, C, workload.SEED_BASE + 4, "cuda")
    g = workload.rng(workload.SEED_BASE + 4)
    A = workload.uniform_u32(g, (C, n))
    Ad = to_dev_u32(A)
    db = qp.Database(D)
    tune.apply(db)   # the variants the benchmark runs
    _step("database and A ready", t0)
    # 4 real LWE queries; the other 252 are uniform words (an LWE query is
    # indistinguishable from uniform, and the answer is checked on its value).
    dr = workload.lwe_draws(g, C, n, 4)
    Q = np.concatenate([lwe_queries(A, dr), workload.uniform_u32(g, (C, B - 4))], axis=1)
    Q = np.ascontiguousarray(Q)
    Qd = to_dev_u32(Q)
    out_d = db.answer_batch(Qd)
    Hd = db.setup_hint(Ad)
    torch.cuda.synchronize()
    _step("batch and hint computed", t0)
    out = to_host_u32(out_d)
    H = to_host_u32(Hd)
    Dh = D.cpu().numpy()
    _step("database, answers and hint copied to the host", t0)
    rows = sample_rows(R, 24, 31)
    assert np.array_equal(out[rows], oracle.answer_batch(Dh[rows], Q))
    _step("batch sampled rows exact", t0)
    hrows = rows[:12]
    assert np.array_equal(H[hrows], oracle.hint(Dh[hrows], A))
    _step("hint sampled rows exact", t0)
    for b in range(4):
        col = int(dr.col[b])
        assert np.array_equal(oracle.lwe_decode(out[:, b], H, dr.s[b]), Dh[:, col])
    _step("4 LWE queries decode on every row", t0)
    assert oracle.freivalds(Dh, Q, out, trials=16, seed=7)
    _step("batch: Freivalds, 16 trials, all rows", t0)
    assert oracle.freivalds(Dh, A, H, trials=16, seed=8)
    _step("hint: Freivalds, 16 trials, all rows", t0)

    # -- refresh 1% of the rows and update the hint incrementally
    m = workload.update_count(R)
    assert m == 1311
    urows = workload.distinct_rows(g, R, m)
    new = workload.db_bytes(g, m, C)
    urows_d = to_dev_u32(urows)
    db.update_rows(urows_d, to_dev_u8(new))
    db.hint_update_rows(urows_d, Ad, Hd)
    torch.cuda.synchronize()
    _step("rows rewritten, hint updated", t0)
    Dh = oracle.update_rows(Dh, urows, new)
    assert np.array_equal(D.cpu().numpy(), Dh)      # the refresh itself, every row
    _step("refreshed database equals the oracle's update", t0)
    H2 = to_host_u32(Hd)
    keep = np.ones(R, dtype=bool)
    keep[urows.astype(np.int64)] = False
    assert np.array_equal(H2[keep], H[keep])        # untouched rows unchanged
    pick = urows[np.random.default_rng(3).choice(m, size=12, replace=False)].astype(np.int64)
    pick.sort()
    assert np.array_equal(H2[pick], oracle.hint(Dh[pick], A))
    _step("updated hint rows exact, other rows untouched", t0)
    assert oracle.freivalds(Dh, A, H2, trials=16, seed=9)
    _step("updated hint: Freivalds, 16 trials, all rows", t0)
    out2 = to_host_u32(db.answer_batch(Qd))
    both = np.unique(np.concatenate([pick, rows]))
    assert np.array_equal(out2[both], oracle.answer_batch(Dh[both], Q))
    for b in range(4):
        col = int(dr.col[b])
        assert np.array_equal(oracle.lwe_decode(out2[:, b], H2, dr.s[b]), Dh[:, col])
    assert oracle.freivalds(Dh, Q, out2, trials=16, seed=10)
    _step("answers after the refresh: sampled rows exact, decodable, Freivalds all rows", t0)
    db.close()
    del D, Dh, Ad, Hd, Qd, out_d
    torch.cuda.empty_cache()
