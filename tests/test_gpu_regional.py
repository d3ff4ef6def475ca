"""The serving workload at its own shapes, checked against the oracle.

Eight regional databases of uneven shapes (4096^2 .. 65536 x 32768 bytes,
4.95 GiB in all) stay resident on the device with the tuned variant table
installed, as the benchmark runs them.  Each database gets its hint and a
pool of real LWE queries (n = 1024, sigma = 6.4) built by the oracle's
client.  The serving loop (batches of up to 64, captured graphs, an
in-flight cap, a 2 GiB admission budget) answers Poisson / Zipf(1.1)
traces -- the batched responses under concurrent demand of Section 5.2 and
Figure 3's end-to-end setting -- plus held bursts that leave as one batch of
each power-of-two size, so every tuned tile of every shape runs inside a
graph.

Checks (tolerance 0: the answers are integers):
* every pool query answered alone through the single-query path equals the
  oracle on 64 sampled rows (the first and last included) and decodes to
  the queried column on every row;
* each hint equals the oracle on sampled rows and passes 16 Freivalds trials
  over all rows;
* every served answer equals the same query answered alone.
"""
import time

import numpy as np
import pytest

import oracle
import workload
from _util import banner, sample_rows, to_dev_u32, to_host_u32

pytestmark = pytest.mark.gpu

POOL = 64            # LWE queries per database
BUDGET = 2 << 30     # admission budget of the serving workload
MAX_BATCH = 64
SLOTS = 3
INFLIGHT = 4


def _step(msg, t0):
    print(f"  [{time.perf_counter() - t0:7.1f}s] {msg}", flush=True)


@pytest.fixture(scope="module")
def regional(gpu):
    import torch
    import paper_2510_03631_amd as qp
    from paper_2510_03631_amd import tune
    t0 = time.perf_counter()
    banner("regional: 8 databases, hints, LWE query pools, answers alone")
    n = workload.LWE_N
    envs = []
    for k, (R, C) in enumerate(workload.SERVING_DBS):
        D = workload.device_db(R, C, workload.SEED_BASE + 30 + k, "cuda")
        db = qp.Database(D)
        tune.apply(db)   # the serving shapes' tuned tiles
        g = workload.rng(workload.SEED_BASE + 60 + k)
        A = workload.uniform_u32(g, (C, n))
        H = to_host_u32(db.setup_hint(to_dev_u32(A)))
        dr = workload.lwe_draws(g, C, n, POOL)
        Q = [oracle.lwe_query(A, dr.s[b], dr.e[b], int(dr.col[b])) for b in range(POOL)]
        alone = [to_host_u32(db.answer(to_dev_u32(q))) for q in Q]
        envs.append(dict(R=R, C=C, D=D, Dh=D.cpu().numpy(), db=db, A=A, H=H, dr=dr,
                         Q=Q, alone=alone))
        _step(f"{R}x{C}: hint, {POOL} queries, answers alone", t0)
    torch.cuda.synchronize()
    yield envs
    for e in envs:
        e["db"].close()
    del envs
    torch.cuda.empty_cache()


def test_regional_hints(regional):
    t0 = time.perf_counter()
    banner("regional hints: sampled rows exact + 16 Freivalds trials over all rows")
    for k, e in enumerate(regional):
        rows = sample_rows(e["R"], 16, 70 + k)
        assert np.array_equal(e["H"][rows], oracle.hint(e["Dh"][rows], e["A"])), k
        assert oracle.freivalds(e["Dh"], e["A"], e["H"], trials=16, seed=80 + k), k
        _step(f"{e['R']}x{e['C']} hint", t0)


def test_regional_alone_vs_oracle(regional):
    t0 = time.perf_counter()
    banner("regional answers alone: 64 sampled rows exact, every row decodes")
    for k, e in enumerate(regional):
        for b in range(POOL):
            a = e["alone"][b]
            rows = sample_rows(e["R"], 64, 1000 * k + b)
            assert np.array_equal(a[rows], oracle.answer(e["Dh"][rows], e["Q"][b])), (k, b)
            col = int(e["dr"].col[b])
            assert np.array_equal(oracle.lwe_decode(a, e["H"], e["dr"].s[b]),
                                  e["Dh"][:, col]), (k, b)
        _step(f"{e['R']}x{e['C']}: {POOL} answers", t0)


def _serve(regional, which, pick, offsets_s):
    from paper_2510_03631_amd.serve import Server
    dbs = [e["db"] for e in regional]
    qs = [regional[d]["Q"][i] for d, i in zip(which, pick)]
    outs = [np.zeros(regional[d]["R"], dtype=np.uint32) for d in which]
    with Server(dbs, max_batch=MAX_BATCH, slots_per_db=SLOTS, mem_budget_bytes=BUDGET,
                max_inflight=INFLIGHT, use_graphs=True) as srv:
        first = srv.replay((np.asarray(offsets_s) * 1e9).astype(np.uint64), which, qs, outs)
        srv.drain()
        lat = srv.latencies(first, len(which))
        st = srv.stats()
    return outs, lat, st


def _check_served(regional, which, pick, outs):
    for j, (d, i) in enumerate(zip(which, pick)):
        assert np.array_equal(outs[j], regional[d]["alone"][i]), (j, int(d), int(i))


@pytest.mark.parametrize("rate,count", [(workload.SERVING_RATE, 600), (300000.0, 2400)])
def test_regional_trace(regional, rate, count):
    """A Poisson trace at the design rate (batches of about one query) and a
    loaded one (batches of tens), Zipf(1.1) over the databases."""
    t0 = time.perf_counter()
    banner(f"regional trace: {count} LWE queries at {rate:.0f} q/s, Zipf(1.1)")
    g = workload.rng(workload.SEED_BASE + 90 + int(rate))
    t = workload.poisson_arrivals(g, rate, 1.5 * count / rate)[:count]
    which = workload.zipf_choice(g, len(regional), len(t))
    pick = g.integers(0, POOL, size=len(t))
    assert len(t) == count and set(which.tolist()) == set(range(len(regional)))
    outs, lat, st = _serve(regional, which, pick, t)
    _step(f"served: {st['batches']} batches, mean {st['batched_queries'] / st['batches']:.2f}", t0)
    assert st["completed"] == count and st["failed"] == 0 and st["rejected"] == 0
    assert (lat > 0).all()
    assert st["peak_inflight_bytes"] <= BUDGET
    if rate > 100000:
        assert st["batched_queries"] / st["batches"] > 4   # batches formed under load
    _check_served(regional, which, pick, outs)
    _step("every served answer equals the query answered alone", t0)


def test_regional_held_batches(regional):
    """Per database, queries held while it is paused leave as one batch on
    resume: sizes 1, 2, 3, 4, 8, 16, 32 and 64 (every power-of-two bucket up
    to the batch cap, and a padded one), each inside its captured graph."""
    from paper_2510_03631_amd.serve import Server
    t0 = time.perf_counter()
    banner("regional held batches of 1..64 on every database")
    dbs = [e["db"] for e in regional]
    g = np.random.default_rng(95)
    sizes = (1, 2, 3, 4, 8, 16, 32, 64)
    with Server(dbs, max_batch=MAX_BATCH, slots_per_db=SLOTS, mem_budget_bytes=BUDGET,
                max_inflight=INFLIGHT, use_graphs=True) as srv:
        for d, e in enumerate(regional):
            for size in sizes:
                pick = g.choice(POOL, size=size, replace=False)
                srv.pause(d)
                s0 = srv.stats()
                outs = [np.zeros(e["R"], dtype=np.uint32) for _ in pick]
                for i, out in zip(pick, outs):
                    srv.submit(d, e["Q"][i], out)
                srv.resume(d)
                srv.drain()
                s1 = srv.stats()
                assert s1["batches"] - s0["batches"] == 1, (d, size)
                assert s1["failed"] == s0["failed"], (d, size)
                for i, out in zip(pick, outs):
                    assert np.array_equal(out, e["alone"][i]), (d, size, int(i))
            _step(f"{e['R']}x{e['C']}: batches of {sizes}", t0)
