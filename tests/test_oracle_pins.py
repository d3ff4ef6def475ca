"""Pins for the CPU oracle: checks against facts fixed outside the oracle.

Each group targets a class of plausible mistakes:
* hand-worked examples (tests/golden/handworked.json) -- wrong sum, wrong
  wrap, transposed operand;
* Python-integer brute force on tiny random and extreme inputs -- any
  indexing, pitch or overflow slip in the C loops;
* closed forms (column selection, scaled column, row sums, all-ones and
  all-0xFF matrices, the 2^31 accumulator case at C = 131072);
* invariants (linearity, batch column = single answer, row permutation,
  hint = batch on A, row update = full recompute);
* the LWE round trip, checked exactly against numpy integer arithmetic
  (a - H s = D e + Delta D[:, i]) and by decoding the queried column;
* decode rounding boundaries.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "handworked.json")
M32 = 1 << 32


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


# ---------------------------------------------------------------- golden
def test_handworked_answer(golden):
    for case in golden["answer"]:
        D = np.array(case["D"], dtype=np.uint8)
        q = np.array(case["q"], dtype=np.uint32)
        assert oracle.answer(D, q).tolist() == case["a"], case["derivation"]


def test_handworked_batch(golden):
    for case in golden["answer_batch"]:
        D = np.array(case["D"], dtype=np.uint8)
        Q = np.array(case["Q"], dtype=np.uint32)
        assert oracle.answer_batch(D, Q).tolist() == case["out"], case["derivation"]


def test_handworked_lwe(golden):
    for case in golden["lwe_round_trip"]:
        A = np.array(case["A"], dtype=np.uint32)
        s = np.array(case["s"], dtype=np.uint32)
        D = np.array(case["D"], dtype=np.uint8)
        q = oracle.lwe_query(A, s, case["e"], case["col"])
        assert q.tolist() == case["q"]
        H = oracle.hint(D, A)
        assert H.tolist() == case["H"]
        a = oracle.answer(D, q)
        assert a.tolist() == case["a"]
        assert oracle.matvec_u32(H, s).tolist() == case["Hs"]
        assert oracle.lwe_decode(a, H, s).tolist() == case["decoded"]


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("seed", range(12))
def test_brute_force_random(seed):
    g = np.random.default_rng(seed)
    R = int(g.integers(1, 18))
    C = int(g.integers(1, 18))
    B = int(g.integers(1, 6))
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    Q = g.integers(0, M32, size=(C, B), dtype=np.uint32)
    assert oracle.answer_batch(D, Q).tolist() == oracle.brute_answer_batch(D.tolist(), Q.tolist())
    for b in range(B):
        assert oracle.answer(D, Q[:, b]).tolist() == oracle.brute_answer(D.tolist(), Q[:, b].tolist())


@pytest.mark.parametrize("dval,qval", [(0, 0), (255, 0xFFFFFFFF), (0x80, 0x80808080),
                                       (255, 0), (0, 0xFFFFFFFF), (1, 0x7FFFFFFF)])
def test_brute_force_extremes(dval, qval):
    R, C, B = 5, 17, 3
    D = np.full((R, C), dval, dtype=np.uint8)
    Q = np.full((C, B), qval, dtype=np.uint32)
    D[0, 0] ^= 0x5A   # break the symmetry so a transposed operand shows
    Q[C - 1, B - 1] ^= 0xDEADBEEF
    assert oracle.answer_batch(D, Q).tolist() == oracle.brute_answer_batch(D.tolist(), Q.tolist())


def test_subset_rows_match_brute():
    g = np.random.default_rng(7)
    D = g.integers(0, 256, size=(13, 9), dtype=np.uint8)
    Q = g.integers(0, M32, size=(9, 4), dtype=np.uint32)
    rows = [12, 0, 5]
    full = oracle.brute_answer_batch(D.tolist(), Q.tolist())
    assert oracle.answer_batch(D, Q, rows=rows).tolist() == [full[r] for r in rows]


# ---------------------------------------------------------------- closed forms
def test_closed_forms():
    g = np.random.default_rng(1)
    R, C = 37, 29
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    for j in (0, 13, C - 1):
        e = np.zeros(C, dtype=np.uint32)
        e[j] = 1
        assert np.array_equal(oracle.answer(D, e), D[:, j].astype(np.uint32))
        e[j] = oracle.DELTA
        assert np.array_equal(oracle.answer(D, e), D[:, j].astype(np.uint32) << 24)
    ones = np.ones(C, dtype=np.uint32)
    assert np.array_equal(oracle.answer(D, ones), D.astype(np.uint64).sum(axis=1).astype(np.uint32))
    q = g.integers(0, M32, size=C, dtype=np.uint32)
    assert not oracle.answer(np.zeros((R, C), np.uint8), q).any()
    expect = (128 * int(q.astype(np.uint64).sum())) % M32
    assert (oracle.answer(np.full((R, C), 0x80, np.uint8), q) == expect).all()


@pytest.mark.parametrize("C", [1, 1000, 131072])
def test_closed_form_all_ff(C):
    D = np.full((3, C), 255, dtype=np.uint8)
    q = np.full(C, 0xFFFFFFFF, dtype=np.uint32)
    assert (oracle.answer(D, q) == (M32 - 255 * C) % M32).all()


def test_accumulator_wrap_closed_forms():
    """C = 131072: sums pass 2^32 many times; the answer is the exact value mod 2^32."""
    C = 131072
    g = np.random.default_rng(3)
    q = g.integers(0, M32, size=C, dtype=np.uint32)
    D = np.zeros((2, C), dtype=np.uint8)
    D[1] = 255
    a = oracle.answer(D, q)
    assert a[0] == 0
    assert a[1] == (255 * int(q.astype(np.uint64).sum())) % M32
    # uint8 x uint8 limbs at their maximum: 0xFF x 0x000000FF over C terms
    qq = np.full(C, 0xFF, dtype=np.uint32)
    assert oracle.answer(D, qq)[1] == (255 * 255 * C) % M32


# ---------------------------------------------------------------- invariants
def test_invariants():
    g = np.random.default_rng(11)
    R, C, B = 23, 41, 6
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    Q = g.integers(0, M32, size=(C, B), dtype=np.uint32)
    out = oracle.answer_batch(D, Q)
    for b in range(B):
        assert np.array_equal(out[:, b], oracle.answer(D, Q[:, b]))
    # linearity over Z/2^32
    x, y = Q[:, 0], Q[:, 1]
    lhs = oracle.answer(D, (x.astype(np.uint64) * 3 + y).astype(np.uint32))
    rhs = (oracle.answer(D, x).astype(np.uint64) * 3 + oracle.answer(D, y)).astype(np.uint32)
    assert np.array_equal(lhs, rhs)
    # row permutation of D permutes the answer
    perm = g.permutation(R)
    assert np.array_equal(oracle.answer(D[perm], x), oracle.answer(D, x)[perm])
    # hint is the batch product on A
    A = g.integers(0, M32, size=(C, 8), dtype=np.uint32)
    assert np.array_equal(oracle.hint(D, A), oracle.answer_batch(D, A))
    # Freivalds accepts the right product and rejects a one-entry error
    assert oracle.freivalds(D, Q, out, trials=8)
    bad = out.copy()
    bad[5, 3] ^= 1 << 31
    assert not oracle.freivalds(D, Q, bad, trials=16)


def test_matvec_u32_against_numpy():
    g = np.random.default_rng(5)
    M = g.integers(0, M32, size=(31, 77), dtype=np.uint32)
    x = g.integers(0, M32, size=77, dtype=np.uint32)
    # numpy's uint64 product wraps mod 2^64, a multiple of 2^32
    ref = (M.astype(np.uint64) @ x.astype(np.uint64)).astype(np.uint32)
    assert np.array_equal(oracle.matvec_u32(M, x), ref)


def test_update_rows_equals_recompute():
    g = np.random.default_rng(9)
    R, C, n = 40, 33, 16
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    A = g.integers(0, M32, size=(C, n), dtype=np.uint32)
    rows = workload.distinct_rows(g, R, 5)
    new = g.integers(0, 256, size=(5, C), dtype=np.uint8)
    D2 = oracle.update_rows(D, rows, new)
    assert np.array_equal(D2[rows], new)
    untouched = np.setdiff1d(np.arange(R), rows)
    assert np.array_equal(D2[untouched], D[untouched])
    H = oracle.hint(D, A)
    H2 = H.copy()
    H2[rows] = oracle.hint(D2, A, rows=rows)
    assert np.array_equal(H2, oracle.hint(D2, A))


# ---------------------------------------------------------------- LWE round trip
def _lwe_case(R, C, n, seed):
    g = workload.rng(seed)
    D = workload.db_bytes(g, R, C)
    A = workload.uniform_u32(g, (C, n))
    dr = workload.lwe_draws(g, C, n, 1)
    return D, A, dr.s[0], dr.e[0], int(dr.col[0])


@pytest.mark.parametrize("R,C,n", [(1024, 1024, 1024), (64, 4096, 256), (300, 77, 32)])
def test_lwe_round_trip_exact(R, C, n):
    D, A, s, e, col = _lwe_case(R, C, n, workload.SEED_BASE)
    q = oracle.lwe_query(A, s, e, col)
    a = oracle.answer(D, q)
    H = oracle.hint(D, A)
    # exact identity over the integers mod 2^32, checked with numpy int64
    De = D.astype(np.int64) @ e.astype(np.int64)
    expect = (De + oracle.DELTA * D[:, col].astype(np.int64)) % M32
    got = (a.astype(np.int64) - oracle.matvec_u32(H, s).astype(np.int64)) % M32
    assert np.array_equal(got, expect)
    assert np.array_equal(oracle.lwe_decode(a, H, s), D[:, col])


def test_decode_rounding_boundaries():
    """Noise in [-2^23, 2^23) decodes to m; +2^23 rounds up to m+1."""
    H = np.zeros((6, 1), dtype=np.uint32)
    s = np.zeros(1, dtype=np.uint32)
    m = np.array([0, 7, 255, 0, 100, 255], dtype=np.int64)
    noise = np.array([(1 << 23) - 1, -(1 << 23), 0, -1, 1 << 23, (1 << 23) - 1])
    a = ((m << 24) + noise) % M32
    dec = oracle.lwe_decode(a.astype(np.uint32), H, s)
    assert dec.tolist() == [0, 7, 255, 0, 101, 255]


# ---------------------------------------------------------------- Chor XOR PIR
def test_chor_handworked():
    # rows 0b0011, 0b0101, 0b1001 as one-word blocks; select rows 0 and 2:
    # 0011 ^ 1001 = 1010
    DB = np.array([[3], [5], [9]], dtype=np.uint32)
    assert oracle.chor_answer(DB, [0b101]).tolist() == [0b1010]
    assert oracle.chor_answer(DB, [0b111]).tolist() == [3 ^ 5 ^ 9]
    assert oracle.chor_answer(DB, [0]).tolist() == [0]


@pytest.mark.parametrize("seed", range(6))
def test_chor_brute_force(seed):
    g = np.random.default_rng(seed)
    r, W = int(g.integers(1, 70)), int(g.integers(1, 5))
    DB = g.integers(0, M32, size=(r, W), dtype=np.uint32)
    q = workload.chor_query_words(g, r, 1)[0]
    sel = oracle.chor_unpack(q, r)
    rows_int = [sum(int(DB[i, w]) << (32 * w) for w in range(W)) for i in range(r)]
    got = oracle.chor_answer(DB, q)
    got_int = sum(int(got[w]) << (32 * w) for w in range(W))
    assert got_int == oracle.brute_chor(rows_int, sel.tolist())
    # packing round trip, and the last word's padding bits stay zero
    assert np.array_equal(oracle.chor_pack(sel), q)


def test_chor_closed_forms_and_linearity():
    g = np.random.default_rng(3)
    r, W = 100, 7
    DB = g.integers(0, M32, size=(r, W), dtype=np.uint32)
    for i in (0, 31, 32, 99):
        e = np.zeros(r, dtype=bool)
        e[i] = True
        assert np.array_equal(oracle.chor_answer(DB, oracle.chor_pack(e)), DB[i])
    allq = oracle.chor_pack(np.ones(r, dtype=bool))
    assert np.array_equal(oracle.chor_answer(DB, allq), np.bitwise_xor.reduce(DB, axis=0))
    q1, q2 = workload.chor_query_words(g, r, 2)
    assert np.array_equal(oracle.chor_answer(DB, q1 ^ q2),
                          oracle.chor_answer(DB, q1) ^ oracle.chor_answer(DB, q2))


@pytest.mark.parametrize("servers", [2, 3, 5])
def test_chor_reconstruction(servers):
    """Shares that XOR to the unit vector of theta: the XOR of the servers'
    responses is row theta (Chor's correctness, Section 5.1)."""
    g = np.random.default_rng(servers)
    r, W, theta = 77, 6, 41
    DB = g.integers(0, M32, size=(r, W), dtype=np.uint32)
    shares = list(workload.chor_shares(g, r, theta, servers))
    e = np.zeros(r, dtype=bool)
    e[theta] = True
    last = oracle.chor_pack(e)
    for s in shares:
        last = last ^ s
    shares.append(last)
    resp = [oracle.chor_answer(DB, s) for s in shares]
    assert np.array_equal(oracle.chor_reconstruct(resp), DB[theta])


# ---------------------------------------------------------------- Goldberg field form
FIELD_PRIMES = (2, 257, 65537, 2147483647, workload.FTR_PRIME)


def test_handworked_field(golden):
    for case in golden["answer_mod"]:
        D = np.array(case["D"], dtype=np.uint8)
        Q = np.array(case["Q"], dtype=np.uint32)
        assert oracle.answer_batch_mod(D, Q, case["p"]).tolist() == case["out"]
        assert oracle.brute_answer_batch_mod(case["D"], case["Q"], case["p"]) == case["out"]


def test_handworked_shamir(golden):
    for case in golden["shamir"]:
        p = case["p"]
        sh = oracle.shamir_shares(case["secret"], case["coeffs"], case["alphas"], p)
        assert sh.tolist() == case["shares"]
        D = np.array(case["D"], dtype=np.uint8)
        resp = [oracle.answer_batch_mod(D, sh[i][:, None], p)[:, 0] for i in range(len(sh))]
        assert [r.tolist() for r in resp] == case["responses"]
        assert oracle.lagrange_weights_at_zero(case["alphas"], p) == case["weights"]
        assert oracle.lagrange_at_zero(case["alphas"], resp, p).tolist() == case["record"]


@pytest.mark.parametrize("seed", range(6))
def test_field_brute_force(seed):
    g = np.random.default_rng(500 + seed)
    R, C, B = (int(x) for x in g.integers(1, 9, size=3))
    p = FIELD_PRIMES[seed % len(FIELD_PRIMES)]
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    Q = workload.uniform_u32(g, (C, B))          # words >= p are taken as integers
    exp = oracle.brute_answer_batch_mod(D.tolist(), Q.tolist(), p)
    assert oracle.answer_batch_mod(D, Q, p).tolist() == exp
    rows = [R - 1, 0]
    assert oracle.answer_batch_mod(D, Q, p, rows=rows).tolist() == [exp[R - 1], exp[0]]
    ent = oracle.answer_mod_entries(D[[R - 1] * B], Q.T, p)
    assert ent.tolist() == exp[R - 1]


def test_field_equals_ring_when_no_reduction():
    # With D Q below both p and 2^32, the field and ring answers are the same
    # integer; the ring oracle is an independent loop.
    g = np.random.default_rng(7)
    D = g.integers(0, 256, size=(20, 64), dtype=np.uint8)
    Q = g.integers(0, 1 << 16, size=(64, 5), dtype=np.uint32)   # D Q < 64 * 255 * 2^16 < 2^31
    assert np.array_equal(oracle.answer_batch_mod(D, Q, workload.FTR_PRIME),
                          oracle.answer_batch(D, Q))


def test_field_closed_forms():
    p = workload.FTR_PRIME
    C = 1000
    D = np.full((3, C), 255, dtype=np.uint8)
    Q = np.full((C, 2), p - 1, dtype=np.uint32)                  # -1 mod p
    assert np.all(oracle.answer_batch_mod(D, Q, p) == (-255 * C) % p)
    # A unit query column returns the selected column of D (the record).
    g = np.random.default_rng(8)
    D = g.integers(0, 256, size=(9, 40), dtype=np.uint8)
    E = np.zeros((40, 3), dtype=np.uint32)
    for b, th in enumerate((0, 17, 39)):
        E[th, b] = 1
    assert np.array_equal(oracle.answer_batch_mod(D, E, p), D[:, [0, 17, 39]].astype(np.uint32))
    # Linearity over Z/p.
    Q1 = workload.uniform_mod(g, (40, 4), p)
    Q2 = workload.uniform_mod(g, (40, 4), p)
    Qs = ((Q1.astype(np.uint64) + Q2) % p).astype(np.uint32)
    lhs = oracle.answer_batch_mod(D, Qs, p).astype(np.uint64)
    rhs = (oracle.answer_batch_mod(D, Q1, p).astype(np.uint64) +
           oracle.answer_batch_mod(D, Q2, p)) % p
    assert np.array_equal(lhs, rhs)


@pytest.mark.parametrize("p", [257, 65537, workload.FTR_PRIME])
def test_lagrange_recovers_constant_term(p):
    g = np.random.default_rng(p % 1000)
    for t in (1, 2, 4):
        coef = [int(c) for c in g.integers(0, p, size=t + 1)]
        coef[-1] = coef[-1] or 1                                 # degree exactly t
        f = lambda x: sum(c * pow(x, k, p) for k, c in enumerate(coef)) % p
        alphas = [int(a) for a in g.choice(np.arange(1, min(p, 5000)), size=t + 1, replace=False)]
        vals = [np.array([f(a)], dtype=np.uint32) for a in alphas]
        assert int(oracle.lagrange_at_zero(alphas, vals, p)[0]) == coef[0]
        # t points of a degree-t polynomial do not determine f(0) (here they
        # miss it unless a 1/p coincidence happens).
        if t >= 1 and p > 1000:
            assert int(oracle.lagrange_at_zero(alphas[:t], vals[:t], p)[0]) != coef[0]


@pytest.mark.parametrize("servers,t", [(3, 1), (5, 2), (6, 4)])
def test_shamir_round_trip_recovers_record(servers, t):
    p = workload.FTR_PRIME
    g = np.random.default_rng(servers * 10 + t)
    R, C = 11, 57                                   # 11 byte positions, 57 records
    D = g.integers(0, 256, size=(R, C), dtype=np.uint8)
    thetas = [3, 0, 56]
    alphas = list(range(1, servers + 1))
    # One share vector per retrieval per server: Q_i is C x len(thetas).
    Qs = np.zeros((servers, C, len(thetas)), dtype=np.uint32)
    for b, th in enumerate(thetas):
        e = np.zeros(C, dtype=np.uint32)
        e[th] = 1
        sh = oracle.shamir_shares(e, workload.uniform_mod(g, (t, C), p), alphas, p)
        Qs[:, :, b] = sh
        assert not np.array_equal(sh[0], e)                    # shares hide e_theta
    resp = [oracle.answer_batch_mod(D, Qs[i], p) for i in range(servers)]
    want = D[:, thetas].astype(np.uint32)
    # Any t + 1 responses reconstruct the records.
    for pick in (list(range(t + 1)), list(range(servers - t - 1, servers))):
        got = oracle.lagrange_at_zero([alphas[i] for i in pick], [resp[i] for i in pick], p)
        assert np.array_equal(got, want)
    # t responses do not.
    got = oracle.lagrange_at_zero(alphas[:t], resp[:t], p)
    assert not np.array_equal(got, want)
