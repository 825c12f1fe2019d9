"""Pins of the CPU oracle against facts fixed outside it (no GPU).

Each test checks the oracle against something the oracle does not compute
itself: published constants and test vectors, closed forms of the
multilinear extension, independent algorithms (doubling, variable-by-variable
folding), brute force on tiny inputs and the protocol's own invariants
(completeness, g(0) + g(1) = claim, degree <= 2, the final-point identity).
"""
import random

import numpy as np
import pytest

import oracle
from oracle import P, eq_table, mle_eval, matrix_mle, partial_eval_rows, partial_eval_cols
from oracle.zkmat import (prove_group, verify_group, FalseStatement, Reject, round_poly, fold,
                          interpolate_quadratic, claim_value, proof_len)
import workloads


def rnd_point(rng, n):
    return [rng.randrange(P) for _ in range(n)]


# ---------------------------------------------------------------- field -----
def test_modulus_is_bls12_381_scalar_field():
    # BLS12 family: r(x) = x^4 - x^2 + 1 with the published BLS12-381 seed.
    x = -0xd201000000010000
    assert P == x ** 4 - x ** 2 + 1
    assert P.bit_length() == 255
    assert (P - 1) % (1 << 32) == 0 and (P - 1) % (1 << 33) != 0  # 2-adicity 32


def test_modulus_is_prime_miller_rabin():
    d, s = P - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41):
        x = pow(a, d, P)
        if x in (1, P - 1):
            continue
        for _ in range(s - 1):
            x = x * x % P
            if x == P - 1:
                break
        else:
            pytest.fail(f"witness {a} shows P composite")


def test_lift_and_encoding():
    assert oracle.lift(-1) == P - 1
    assert oracle.lift(-(1 << 15)) == P - (1 << 15)
    assert oracle.enc(1) == b"\x01" + b"\x00" * 31
    assert oracle.dec(oracle.enc(P - 1)) == P - 1
    with pytest.raises(ValueError):
        oracle.dec(P.to_bytes(32, "little"))
    assert oracle.inv(2) * 2 % P == 1
    for x in (2, 3, 12345, P - 1, 2**200 + 7):
        assert oracle.inv(x) == pow(x, P - 2, P)   # Fermat's little theorem


# ---------------------------------------------------------------- hash ------
def test_sha256_fips_180_4_vectors():
    assert oracle.sha256(b"abc").hex() == \
        "ba7816bf8f01cfea414140de5dae2223b00361a396177a9cb410ff61f20015ad"
    assert oracle.sha256(b"abcdbcdecdefdefgefghfghighijhijkijkljklmklmnlmnomnopnopq").hex() == \
        "248d6a61d20638b8e5c026930c3e6039a33ce45964ff2167f6ecedd419db06c1"
    assert oracle.sha256(b"").hex() == \
        "e3b0c44298fc1c149afbf4c8996fb92427ae41e4649b934ca495991b7852b855"


def test_transcript_rejection_sampling_is_exercised():
    tr = oracle.Transcript(7, 3, [(4, 8, 2)])
    seen_reject = 0
    for _ in range(200):
        st = tr.state
        x = tr.squeeze(b"r")
        assert 0 <= x < P
        first = int.from_bytes(oracle.sha256(st + b"r" + (0).to_bytes(4, "little")), "little")
        if (first & ((1 << 255) - 1)) >= P:
            seen_reject += 1
    # acceptance probability is p / 2^255 ~ 0.906: about 19 of 200 need a retry
    assert 3 <= seen_reject <= 45


def test_transcript_binds_every_input():
    base = oracle.Transcript(1, 0, [(64, 128, 32)]).squeeze(b"u")
    assert oracle.Transcript(2, 0, [(64, 128, 32)]).squeeze(b"u") != base
    assert oracle.Transcript(1, 1, [(64, 128, 32)]).squeeze(b"u") != base
    assert oracle.Transcript(1, 0, [(64, 128, 16)]).squeeze(b"u") != base
    assert oracle.Transcript(1, 0, [(64, 128, 32)]).squeeze(b"v") != base


# ---------------------------------------------------------------- MLE -------
@pytest.mark.parametrize("n", [0, 1, 3, 5])
def test_eq_partition_of_unity_and_boolean_points(n):
    rng = random.Random(n)
    x = rnd_point(rng, n)
    assert sum(eq_table(x)) % P == 1
    for j in range(1 << n):
        bits = [(j >> (n - 1 - t)) & 1 for t in range(n)]
        assert eq_table(bits) == [1 if i == j else 0 for i in range(1 << n)]


def eq_by_doubling(x):
    """Independent construction: start from [1]; each new variable splits every
    entry e into (e (1 - x_j), e x_j) appended as the next lower bit."""
    t = [1]
    for xj in x:
        t = [v for e in t for v in (e * (1 - xj) % P, e * xj % P)]
    return t


def mle_by_folding(values, x):
    """Independent evaluation: fix the variables one at a time, leading first."""
    v = list(values) + [0] * ((1 << len(x)) - len(values))
    for xj in x:
        h = len(v) // 2
        v = [(v[t] + xj * (v[t + h] - v[t])) % P for t in range(h)]
    return v[0]


@pytest.mark.parametrize("n", [1, 2, 4, 6])
def test_eq_table_matches_doubling_and_folding(n):
    rng = random.Random(100 + n)
    x = rnd_point(rng, n)
    assert eq_table(x) == eq_by_doubling(x)
    vals = [rng.randrange(-1000, 1000) for _ in range((1 << n) - rng.randrange(2))]
    assert mle_eval(vals, x) == mle_by_folding([v % P for v in vals], x)
    # boolean points give the values back (Lagrange basis property)
    for i in range(len(vals)):
        bits = [(i >> (n - 1 - t)) & 1 for t in range(n)]
        assert mle_eval(vals, bits) == vals[i] % P


def test_matrix_mle_closed_forms():
    rng = random.Random(5)
    n = 3
    D = 1 << n
    u, v = rnd_point(rng, n), rnd_point(rng, n)
    identity = np.eye(D, dtype=np.int64)
    expect = 1
    for uj, vj in zip(u, v):
        expect = expect * (uj * vj + (1 - uj) * (1 - vj)) % P
    assert matrix_mle(identity, u, v) == expect
    assert claim_value(identity, u, v) == expect
    # all ones with a full power-of-two row count: a[k] = sum_i eq(u, i) = 1
    ones = np.ones((D, 5), dtype=np.int64)
    assert partial_eval_rows(ones, u) == [1] * 5 + [0] * 3
    # rank one: A = x y^T  ->  a[k] = (eq_u . x) y_k
    xs = np.array([rng.randrange(-99, 99) for _ in range(D)], dtype=np.int64)
    ys = np.array([rng.randrange(-99, 99) for _ in range(6)], dtype=np.int64)
    A = np.outer(xs, ys)
    eu = eq_table(u)
    s = sum(e * int(xv) for e, xv in zip(eu, xs)) % P
    assert partial_eval_rows(A, u) == [s * int(y) % P for y in ys] + [0, 0]
    bt = partial_eval_cols(A.T, u)
    assert bt == [s * int(y) % P for y in ys] + [0, 0]


def test_partial_evals_against_brute_force():
    rng = random.Random(11)
    M = np.array([[rng.randrange(-(1 << 15), 1 << 15) for _ in range(5)] for _ in range(3)],
                 dtype=np.int64)
    x = rnd_point(rng, 2)
    y = rnd_point(rng, 3)
    a = partial_eval_rows(M, x)
    b = partial_eval_cols(M, y)
    assert len(a) == 8 and len(b) == 4
    for k in range(8):
        wk = [(k >> (2 - t)) & 1 for t in range(3)]
        assert a[k] == matrix_mle(M, x, wk)
    for i in range(4):
        wi = [(i >> (1 - t)) & 1 for t in range(2)]
        assert b[i] == matrix_mle(M, wi, y)
    r = rnd_point(rng, 3)
    assert mle_by_folding(a, r) == matrix_mle(M, x, r)


def test_exact_matmul_matches_integer_definition():
    rng = np.random.default_rng(0)
    a = rng.integers(-(1 << 15), 1 << 15, size=(5, 7), dtype=np.int16)
    b = rng.integers(-(1 << 15), 1 << 15, size=(7, 3), dtype=np.int16)
    c = workloads.exact_matmul(a, b)
    for i in range(5):
        for j in range(3):
            assert c[i, j] == sum(int(a[i, k]) * int(b[k, j]) for k in range(7))
    # the float64 route (taken above 2^22 MACs) is exact: compare with int64 matmul
    a = rng.integers(-(1 << 15), 1 << 15, size=(256, 512), dtype=np.int16)
    b = rng.integers(-(1 << 15), 1 << 15, size=(512, 64), dtype=np.int16)
    assert np.array_equal(workloads.exact_matmul(a, b), a.astype(np.int64) @ b.astype(np.int64))


def test_requant_rounding():
    z = np.array([0, 2047, 2048, -2048, -2049, 4096 * 40000, -4096 * 40000], dtype=np.int64)
    assert workloads.requant(z).tolist() == [0, 0, 1, 0, -1, 32767, -32768]


# ---------------------------------------------------------------- sumcheck --
def test_lagrange_interpolation_on_012():
    rng = random.Random(3)
    for _ in range(10):
        c0, c1, c2, r = (rng.randrange(P) for _ in range(4))
        q = lambda X: (c0 + c1 * X + c2 * X * X) % P  # noqa: E731
        assert interpolate_quadratic(q(0), q(1), q(2), r) == q(r)


def test_round_poly_identities():
    rng = random.Random(4)
    a = [rng.randrange(P) for _ in range(16)]
    b = [rng.randrange(P) for _ in range(16)]
    g0, g1, g2 = round_poly(a, b)
    assert (g0 + g1) % P == sum(x * y for x, y in zip(a, b)) % P
    # degree <= 2: g(3) from the definition equals the extrapolation
    h = 8
    g3 = sum((a[t] + 3 * (a[t + h] - a[t])) * (b[t] + 3 * (b[t + h] - b[t])) for t in range(h)) % P
    assert interpolate_quadratic(g0, g1, g2, 3) == g3
    r = rng.randrange(P)
    assert interpolate_quadratic(g0, g1, g2, r) == \
        sum(x * y for x, y in zip(fold(a, r), fold(b, r))) % P


SHAPES = [
    [(4, 8, 2)], [(3, 5, 7)], [(1, 1, 1)], [(1, 6, 1)], [(5, 1, 3)], [(2, 2, 9)],
    [(4, 8, 4), (4, 3, 4)], [(3, 16, 2), (3, 1, 2), (3, 5, 2)],
]


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("trans", [(False, False), (True, True)])
def test_completeness_and_witness_final_point(dims, trans):
    g = workloads.tiny_random_group(sum(map(sum, dims)) + trans[0], dims, trans=trans)
    prods = [(p.opA(), p.opB()) for p in g.products]
    proof, state, det = prove_group(prods, g.C, 9, 2)
    assert len(proof) == proof_len(g.shapes)
    res = verify_group(proof, g.shapes, 9, 2, witness=(prods, g.C))
    assert res["state"] == state
    # the final claims are A~(u, r) and B~(r, v), by the definition
    for (A, B), rvec, (af, bf) in zip(prods, det["r"], det["finals"]):
        assert matrix_mle(A, det["u"], rvec) == af
        assert matrix_mle(B, rvec, det["v"]) == bf
    assert matrix_mle(g.C, det["u"], det["v"]) == det["c"]


def test_every_single_element_tamper_is_rejected():
    g = workloads.tiny_random_group(21, [(4, 8, 4), (4, 2, 4)])
    prods = [(p.opA(), p.opB()) for p in g.products]
    proof, _, _ = prove_group(prods, g.C, 5, 0)
    for pos in range(0, len(proof), 32):
        x = int.from_bytes(proof[pos:pos + 32], "little")
        bad = proof[:pos] + ((x + 1) % P).to_bytes(32, "little") + proof[pos + 32:]
        with pytest.raises(Reject):
            verify_group(bad, g.shapes, 5, 0)
    with pytest.raises(Reject):
        verify_group(proof, g.shapes, 6, 0)   # another seed: other challenges
    with pytest.raises(Reject):
        verify_group(proof[:-32], g.shapes, 5, 0)
    with pytest.raises(Reject):
        verify_group(proof[:-32] + P.to_bytes(32, "little"), g.shapes, 5, 0)


def test_false_statement_is_refused():
    g = workloads.tiny_random_group(3, [(8, 8, 8)])
    prods = [(p.opA(), p.opB()) for p in g.products]
    bad = g.C.copy()
    bad[7, 0] += 1
    with pytest.raises(FalseStatement):
        prove_group(prods, bad, 1, 0)
    # a transposed operand is a different statement
    with pytest.raises(FalseStatement):
        prove_group([(prods[0][0], prods[0][1].T.copy())], g.C, 1, 0)


def test_wrong_witness_rejected_by_evaluation():
    g = workloads.tiny_random_group(8, [(4, 4, 4)])
    prods = [(p.opA(), p.opB()) for p in g.products]
    proof, _, _ = prove_group(prods, g.C, 1, 0)
    A2 = prods[0][0].copy()
    A2[0, 0] += 1
    with pytest.raises(Reject):
        verify_group(proof, g.shapes, 1, 0, witness=([(A2, prods[0][1])], g.C))
