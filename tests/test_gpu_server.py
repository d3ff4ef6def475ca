"""Serving loop: continuous batching, memory-budget admission, graph replay.

Each query's answer must be the same alone and in the mix (tolerance 0: the
results are integers), and equal to the oracle's.
"""
import numpy as np
import pytest

import oracle
import workload
from _util import banner, to_dev_u32, to_dev_u8, to_host_u32

pytestmark = pytest.mark.gpu
M32 = 1 << 32

SHAPES = [(512, 1024), (1000, 2048), (2048, 512), (300, 4096)]


@pytest.fixture(scope="module")
def env(gpu):
    import paper_2510_03631_amd as qp
    g = np.random.default_rng(4242)
    Ds = [g.integers(0, 256, size=s, dtype=np.uint8) for s in SHAPES]
    dbs = [qp.Database(to_dev_u8(D)) for D in Ds]
    queries = [[g.integers(0, M32, size=s[1], dtype=np.uint32) for _ in range(24)] for s in SHAPES]
    expected = [[oracle.answer(D, q) for q in qs] for D, qs in zip(Ds, queries)]
    yield dict(qp=qp, Ds=Ds, dbs=dbs, queries=queries, expected=expected, g=g)
    for db in dbs:
        db.close()


def _mixed_order(env, seed):
    g = np.random.default_rng(seed)
    order = [(d, i) for d in range(len(SHAPES)) for i in range(24)]
    g.shuffle(order)
    return order


@pytest.mark.parametrize("use_graphs", [True, False])
def test_alone_equals_in_mix(env, use_graphs):
    from paper_2510_03631_amd.serve import Server
    banner(f"server alone == mix, graphs={use_graphs}")
    dbs, queries, expected = env["dbs"], env["queries"], env["expected"]
    # alone: each query by itself through the single-query entry point
    alone = [[to_host_u32(db.answer(to_dev_u32(q))) for q in qs] for db, qs in zip(dbs, queries)]
    for d in range(len(SHAPES)):
        for i in range(24):
            assert np.array_equal(alone[d][i], expected[d][i])
    with Server(dbs, max_batch=16, slots_per_db=2, use_graphs=use_graphs) as srv:
        outs = {}
        for rep in range(3):   # replays of the captured graphs, eager work between
            order = _mixed_order(env, rep)
            for d, i in order:
                outs[(rep, d, i)] = np.zeros(SHAPES[d][0], dtype=np.uint32)
                srv.submit(d, queries[d][i], outs[(rep, d, i)])
            srv.drain()
            _ = to_host_u32(dbs[0].answer(to_dev_u32(queries[0][0])))   # eager work between
        st = srv.stats()
    for (rep, d, i), out in outs.items():
        assert np.array_equal(out, alone[d][i]), (rep, d, i)
    assert st["completed"] == 3 * 24 * len(SHAPES) and st["failed"] == 0
    assert st["batches"] <= st["completed"]


def test_burst_forms_batches(env):
    from paper_2510_03631_amd.serve import Server
    banner("server burst batching")
    dbs, queries, expected = env["dbs"], env["queries"], env["expected"]
    with Server(dbs, max_batch=32, slots_per_db=1) as srv:
        outs = []
        for i in range(24):
            out = np.zeros(SHAPES[1][0], dtype=np.uint32)
            srv.submit(1, queries[1][i], out)
            outs.append(out)
        srv.drain()
        st = srv.stats()
    for i in range(24):
        assert np.array_equal(outs[i], expected[1][i])
    assert st["batches"] < 24          # arrivals during a running batch were batched


@pytest.mark.parametrize("max_inflight", [1, 0])
def test_inflight_cap(env, max_inflight):
    # One batch on the device at a time (everything else waits in the
    # queues, oldest database first), or no cap beyond the slots: the answers
    # are the same either way.
    from paper_2510_03631_amd.serve import Server
    banner(f"server max_inflight={max_inflight}")
    dbs, queries, expected = env["dbs"], env["queries"], env["expected"]
    with Server(dbs, max_batch=16, slots_per_db=2, max_inflight=max_inflight) as srv:
        outs = {}
        for d, i in _mixed_order(env, 11):
            outs[(d, i)] = np.zeros(SHAPES[d][0], dtype=np.uint32)
            srv.submit(d, queries[d][i], outs[(d, i)])
        srv.drain()
        st = srv.stats()
    for (d, i), out in outs.items():
        assert np.array_equal(out, expected[d][i]), (d, i)
    assert st["completed"] == 24 * len(SHAPES) and st["failed"] == 0
    if max_inflight == 1:
        assert st["batches"] < st["completed"]   # queued work left in batches


@pytest.mark.parametrize("use_graphs", [True, False])
def test_held_queue_leaves_as_one_batch(env, use_graphs):
    # Queries queued while their database is paused leave as one batch of
    # 16 on resume: the size whose copies run as plain stream copies around
    # the graph of kernels (batches of 8 or more); the answers equal the
    # oracle's, twice in a row.
    from paper_2510_03631_amd.serve import Server
    banner(f"server held queue -> one batch of 16, graphs={use_graphs}")
    dbs, queries, expected = env["dbs"], env["queries"], env["expected"]
    with Server(dbs, max_batch=16, slots_per_db=2, use_graphs=use_graphs) as srv:
        for rep in range(2):
            srv.pause(2)
            s0 = srv.stats()
            outs = []
            for i in range(16):
                outs.append(np.zeros(SHAPES[2][0], dtype=np.uint32))
                srv.submit(2, queries[2][i + rep], outs[-1])
            srv.resume(2)
            srv.drain()
            s1 = srv.stats()
            assert s1["batches"] - s0["batches"] == 1, rep
            for i in range(16):
                assert np.array_equal(outs[i], expected[2][i + rep]), (rep, i)


def test_memory_budget_admission(env):
    from paper_2510_03631_amd.serve import Server
    banner("server tiny memory budget")
    dbs, queries, expected = env["dbs"], env["queries"], env["expected"]
    # room for one single-query batch of the largest footprint, no more
    budget = max((R + C) * 4 + db.workspace_bytes(0) for (R, C), db in zip(SHAPES, dbs)) + 1024
    with Server(dbs, max_batch=16, slots_per_db=2, mem_budget_bytes=budget) as srv:
        outs = {}
        for d, i in _mixed_order(env, 7):
            outs[(d, i)] = np.zeros(SHAPES[d][0], dtype=np.uint32)
            srv.submit(d, queries[d][i], outs[(d, i)])
        srv.drain()
        st = srv.stats()
    assert st["peak_inflight_bytes"] <= budget
    for (d, i), out in outs.items():
        assert np.array_equal(out, expected[d][i])


def test_budget_too_small_and_queue_full(env):
    from paper_2510_03631_amd.serve import Server
    qp = env["qp"]
    banner("server admission errors")
    with pytest.raises(qp.PirError) as e:
        Server(env["dbs"], mem_budget_bytes=1024)
    assert e.value.status == 3
    db = env["dbs"][3]
    with Server([db], max_batch=1, slots_per_db=1, max_queue=2) as srv:
        statuses = []
        for i in range(40):
            try:
                srv.submit(0, env["queries"][3][i % 24])
                statuses.append(0)
            except qp.PirError as err:
                statuses.append(err.status)
        srv.drain()
        st = srv.stats()
    assert 7 in statuses and st["rejected"] == statuses.count(7)
    assert st["completed"] == statuses.count(0)


def test_pause_update_resume(env):
    from paper_2510_03631_amd.serve import Server
    qp = env["qp"]
    banner("server pause / refresh / resume")
    g = np.random.default_rng(5)
    R, C = 700, 1536
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    q = g.integers(0, M32, size=C, dtype=np.uint32)
    rows = workload.distinct_rows(g, R, 20)
    new = g.integers(0, 256, size=(20, C), dtype=np.uint8)
    with qp.Database(to_dev_u8(D)) as db, Server([db], max_batch=8) as srv:
        before = np.zeros(R, dtype=np.uint32)
        srv.wait(srv.submit(0, q, before))
        srv.pause(0)
        db.update_rows(to_dev_u32(rows), to_dev_u8(new))
        import torch
        torch.cuda.synchronize()
        srv.resume(0)
        after = np.zeros(R, dtype=np.uint32)
        srv.wait(srv.submit(0, q, after))
    assert np.array_equal(before, oracle.answer(D, q))
    assert np.array_equal(after, oracle.answer(oracle.update_rows(D, rows, new), q))


def test_open_loop_replay(env):
    from paper_2510_03631_amd.serve import Server
    banner("server open-loop replay")
    dbs, queries, expected = env["dbs"], env["queries"], env["expected"]
    g = np.random.default_rng(11)
    t = workload.poisson_arrivals(g, 4000.0, 0.25)
    which = workload.zipf_choice(g, len(SHAPES), len(t))
    pick = g.integers(0, 24, size=len(t))
    qs = [queries[d][i] for d, i in zip(which, pick)]
    outs = [np.zeros(SHAPES[d][0], dtype=np.uint32) for d in which]
    with Server(dbs, max_batch=64, slots_per_db=2) as srv:
        first = srv.replay((t * 1e9).astype(np.uint64), which, qs, outs)
        srv.drain()
        lat = srv.latencies(first, len(t))
        st = srv.stats()
    assert st["completed"] == len(t) and st["failed"] == 0
    assert (lat > 0).all()
    assert st["p50_ns"] <= st["p99_ns"] <= st["max_ns"]
    for k, (d, i) in enumerate(zip(which, pick)):
        assert np.array_equal(outs[k], expected[d][i]), k


def test_narrow_variants_in_graphs(env):
    """The narrow-layout kernels inside captured graphs: every database
    serves batches of up to 4 / 8 / 16 with them, replayed twice with eager
    work between, and every answer equals the oracle's."""
    from paper_2510_03631_amd.serve import Server
    banner("server with narrow variants in graphs")
    dbs, queries, expected = env["dbs"], env["queries"], env["expected"]
    chosen = {4: "narrow_128x32_k128_s6", 8: "narrow_256x32_k128_s4", 16: "narrow_256x64_k128_s4"}
    try:
        for db in dbs:
            for b, name in chosen.items():
                db.set_variant(b, name)
        # One slot per database and bursts per database, so batches of
        # several queries form (and reach the narrow tiles).
        with Server(dbs, max_batch=16, slots_per_db=1, use_graphs=True) as srv:
            outs = {}
            for rep in range(2):
                for d in range(len(SHAPES)):
                    for i in range(24):
                        outs[(rep, d, i)] = np.zeros(SHAPES[d][0], dtype=np.uint32)
                        srv.submit(d, queries[d][i], outs[(rep, d, i)])
                srv.drain()
                _ = to_host_u32(dbs[1].answer(to_dev_u32(queries[1][0])))   # eager work between
            st = srv.stats()
    finally:
        for db in dbs:
            for b in chosen:
                db.set_variant(b, 0)
    for (rep, d, i), out in outs.items():
        assert np.array_equal(out, expected[d][i]), (rep, d, i)
    assert st["failed"] == 0 and st["batches"] < st["completed"]


def test_paused_queue_drain_and_destroy(env):
    """A drain while a paused database holds queued requests returns BUSY
    instead of blocking; destroying the server resumes the database and
    finishes them (answers equal the oracle's)."""
    from paper_2510_03631_amd.serve import Server
    qp = env["qp"]
    banner("server: drain while paused, destroy finishes held requests")
    dbs, queries, expected = env["dbs"], env["queries"], env["expected"]
    srv = Server(dbs, max_batch=16, slots_per_db=2)
    try:
        srv.pause(1)
        outs = []
        for i in range(5):
            outs.append(np.zeros(SHAPES[1][0], dtype=np.uint32))
            srv.submit(1, queries[1][i], outs[-1])
        other = np.zeros(SHAPES[0][0], dtype=np.uint32)
        srv.wait(srv.submit(0, queries[0][0], other))   # other databases keep serving
        with pytest.raises(qp.PirError) as e:
            srv.drain()
        assert e.value.status == 7
        st = srv.stats()
        assert st["completed"] == 1 and st["device_bytes"] > 0
    finally:
        srv.close()   # resumes database 1 and finishes its five requests
    assert np.array_equal(other, expected[0][0])
    for i in range(5):
        assert np.array_equal(outs[i], expected[1][i]), i
