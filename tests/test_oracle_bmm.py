"""Pins of the per-head batched matmul oracle (oracle/bmm.py) against facts fixed outside it (no GPU).

The batched sumcheck proves C_h = A_h B_h for every head h of an attention
layer (Sec. III-A, eq. (att)) with one sumcheck over (head, inner) variables.
Its pins:
  * with one head it is byte for byte the plain matmul sumcheck of
    eq. (zk-mle-matmul) at the same point (the already pinned zkMat oracle);
  * its claim is the eq(rho, .)-weighted sum of the per-head zkMat claims,
    and the 3-D MLE reduces to the matrix MLE at Boolean head points and to
    the entries at Boolean points (eq. (MLE) is the Lagrange basis);
  * perfect completeness with the witness checked by direct evaluation;
  * every single-element tamper of a proof is rejected, false statements are
    refused;
  * each head round's polynomial has degree 3 and each inner round's degree
    2: the value at X = 4 (resp. 3), computed from the definition of the
    round sum, equals the extrapolation from the sent values;
  * planted mistakes (dropped eq(rho, h) weight, quadratic interpolation of a
    head round, LSB-first head bits, a swapped fold) are caught.
"""
import random

import numpy as np
import pytest

import oracle.bmm as bmm
import oracle.mle as mle
import workloads
from oracle import P, enc
from oracle.mle import eq_basis, bits_msb_first, eq_table, num_vars, partial_eval_rows, partial_eval_cols
from oracle.zkmat import FalseStatement, Reject, claim_value, prove_group_at, matrix_mle

CASES = [
    dict(H=3, d0=5, d1=7, d2=6, transA=True, b_cols=True, c_cols=True),
    dict(H=4, d0=4, d1=8, d2=2),
    dict(H=2, d0=3, d1=1, d2=5, a_cols=True),
    dict(H=5, d0=1, d1=4, d2=1, transB=True),
    dict(H=8, d0=2, d1=2, d2=4, transA=True, transB=True, a_cols=True, b_cols=True),
    dict(H=1, d0=6, d1=9, d2=3),
]


def _case(i):
    kw = dict(CASES[i])
    return workloads.tiny_head_batch(i + 1, kw.pop("H"), kw.pop("d0"), kw.pop("d1"), kw.pop("d2"), **kw)


def _wit(b):
    return (b.opA_heads(), b.opB_heads(), b.C_heads())


@pytest.mark.parametrize("i", range(len(CASES)))
def test_complete_with_witness(i):
    b = _case(i)
    proof, state, det = bmm.prove_batch(b, 17)
    H, d0, d1, d2 = b.dims
    assert len(proof) == bmm.proof_len(H, d1)
    res = bmm.verify(proof, H, d0, d1, d2, 17, b.group_id, witness=_wit(b))
    assert res["state"] == state


@pytest.mark.parametrize("shape", [(6, 9, 3), (4, 8, 4), (1, 1, 1), (3, 2, 5)])
def test_one_head_is_the_plain_matmul_sumcheck(shape):
    # H = 1 has no head variables; the proof must be the zkMat proof of the
    # same product at the same (u, v), continuing the same transcript
    d0, d1, d2 = shape
    b = workloads.tiny_head_batch(5, 1, d0, d1, d2)
    proof, state, det = bmm.prove_batch(b, 3)
    tr = bmm.transcript(3, b.group_id, 1, d0, d1, d2)
    rho, u, v = bmm.challenges(tr, 1, d0, d2)
    assert rho == []
    expect, _ = prove_group_at([(b.opA_heads()[0], b.opB_heads()[0])], b.C_heads()[0], tr, u, v)
    assert proof == expect
    assert state == tr.state


def test_claim_is_the_weighted_sum_of_head_claims():
    rng = random.Random(2)
    b = _case(0)
    H, d0, d1, d2 = b.dims
    rho, u, v = [[rng.randrange(P) for _ in range(n)] for n in (num_vars(H), num_vars(d0), num_vars(d2))]
    expect = sum(eq_basis(rho, bits_msb_first(k, len(rho))) * claim_value(C, u, v)
                 for k, C in enumerate(b.C_heads())) % P
    assert bmm.tensor_mle(b.C_heads(), rho, u, v) == expect


def test_tensor_mle_at_boolean_points():
    b = _case(1)
    Cs = b.C_heads()
    H, d0, _, d2 = b.dims
    nh, n0, n2 = num_vars(H), num_vars(d0), num_vars(d2)
    rng = random.Random(3)
    u, v = [rng.randrange(P) for _ in range(n0)], [rng.randrange(P) for _ in range(n2)]
    for k in range(H):
        # Boolean head point: the head's own matrix MLE
        assert bmm.tensor_mle(Cs, bits_msb_first(k, nh), u, v) == matrix_mle(Cs[k], u, v)
        for i in range(d0):
            for j in range(d2):
                got = bmm.tensor_mle(Cs, bits_msb_first(k, nh), bits_msb_first(i, n0), bits_msb_first(j, n2))
                assert got == int(Cs[k][i, j]) % P
    # a padding head (index >= H) is zero
    b3 = _case(0)   # H = 3, padded to 4
    assert bmm.tensor_mle(b3.C_heads(), [1, 1], [0] * num_vars(5), [0] * num_vars(6)) == 0


@pytest.mark.parametrize("i", [0, 2, 4])
def test_every_single_element_tamper_is_rejected(i):
    b = _case(i)
    proof, _, _ = bmm.prove_batch(b, 23)
    H, d0, d1, d2 = b.dims
    for pos in range(0, len(proof), 32):
        x = int.from_bytes(proof[pos:pos + 32], "little")
        bad = proof[:pos] + enc((x + 1) % P) + proof[pos + 32:]
        with pytest.raises(Reject):
            bmm.verify(bad, H, d0, d1, d2, 23, b.group_id, witness=_wit(b))
    with pytest.raises(Reject):
        bmm.verify(proof[:-32], H, d0, d1, d2, 23, b.group_id)
    with pytest.raises(Reject):   # another seed's transcript
        bmm.verify(proof, H, d0, d1, d2, 24, b.group_id)


def test_false_statement_refused():
    b = _case(1)
    Cs = [c.copy() for c in b.C_heads()]
    Cs[2][1, 0] += 1
    with pytest.raises(FalseStatement):
        bmm.prove(b.opA_heads(), b.opB_heads(), Cs, 5, 0)
    # a head's product swapped for another head's: also false
    Cs = list(b.C_heads())
    Cs[0], Cs[1] = Cs[1], Cs[0]
    with pytest.raises(FalseStatement):
        bmm.prove(b.opA_heads(), b.opB_heads(), Cs, 5, 0)


def _tables(b, rho, u, v):
    """E, a, b over (h, w) from the definitions (eq table and partial
    evaluations), head index most significant."""
    H, d0, d1, d2 = b.dims
    L1 = 1 << num_vars(d1)
    er = eq_table(rho)
    E, a, bb = [], [], []
    for k in range(1 << len(rho)):
        E += [er[k]] * L1
        if k < H:
            a += partial_eval_rows(b.opA_heads()[k], u)
            bb += partial_eval_cols(b.opB_heads()[k], v)
        else:
            a += [0] * L1
            bb += [0] * L1
    return E, a, bb


@pytest.mark.parametrize("i", [0, 1, 4])
def test_round_polynomial_degrees(i):
    # the round sum at X is sum_t prod over the three tables of the line
    # x_t + X (x_{t+h} - x_t); beyond the sent points it must agree with the
    # extrapolation of degree 3 (head rounds) or 2 (inner rounds)
    b = _case(i)
    H, d0, d1, d2 = b.dims
    proof, _, det = bmm.prove_batch(b, 31)
    nh = num_vars(H)
    E, a, bb = _tables(b, det["rho"], det["u"], det["v"])
    for rd, (g, r) in enumerate(zip(det["rounds"], det["r"])):
        h = len(a) // 2
        X = len(g)     # first point not sent
        s = 0
        for t in range(h):
            s += ((E[t] + X * (E[t + h] - E[t])) * (a[t] + X * (a[t + h] - a[t]))
                  * (bb[t] + X * (bb[t + h] - bb[t])))
        assert len(g) == (4 if rd < nh else 3)
        assert s % P == bmm.lagrange_eval(g, X)
        E = [(E[t] + r * (E[t + h] - E[t])) % P for t in range(h)]
        a = [(a[t] + r * (a[t + h] - a[t])) % P for t in range(h)]
        bb = [(bb[t] + r * (bb[t + h] - bb[t])) % P for t in range(h)]


def test_lagrange_eval_matches_numpy_polyfit():
    # an independent route: the cubic through four integer points, fitted
    # exactly with numpy in floating point on small integers
    xs = np.arange(4, dtype=np.float64)
    coef = np.array([3.0, -2.0, 5.0, 7.0])   # 3x^3 - 2x^2 + 5x + 7
    ys = np.polyval(coef, xs)
    for r in (4, 9, -3):
        assert bmm.lagrange_eval([int(y) for y in ys], r % P) == int(np.polyval(coef, r)) % P


# ----------------------------------------------------- planted mistakes --
def _pins_hold() -> bool:
    try:
        for i in (0, 1, 4):
            b = _case(i)
            proof, _, _ = bmm.prove_batch(b, 7)
            bmm.verify(proof, *b.dims, 7, b.group_id, witness=_wit(b))
        b = workloads.tiny_head_batch(5, 1, 4, 8, 2)
        proof, _, _ = bmm.prove_batch(b, 3)
        tr = bmm.transcript(3, 0, 1, 4, 8, 2)
        _, u, v = bmm.challenges(tr, 1, 4, 2)
        expect, _ = prove_group_at([(b.opA_heads()[0], b.opB_heads()[0])], b.C_heads()[0], tr, u, v)
        if proof != expect:
            return False
    except (Reject, FalseStatement, AssertionError, ValueError, IndexError):
        return False
    return True


_orig_line = bmm._line
_orig_lagrange = bmm.lagrange_eval
_orig_eq_basis = mle.eq_basis


def _line_swapped(x, h, X):
    return [(x[t + h] + X * (x[t] - x[t + h])) % P for t in range(h)]


def _lagrange_quadratic(gs, r):
    return _orig_lagrange(list(gs)[:3], r)


def _tensor_mle_lsb(Ms, h, x, y):
    return _orig_tensor_mle(Ms, list(reversed(h)), x, y)


def _tensor_mle_no_head_weight(Ms, h, x, y):
    return sum(matrix_mle(M, x, y) for M in Ms) % P


_orig_tensor_mle = bmm.tensor_mle

MUTATIONS = [
    ("fold weights swapped", [(bmm, "_line", _line_swapped)]),
    ("head rounds interpolated as quadratics", [(bmm, "lagrange_eval", _lagrange_quadratic)]),
    ("head bits least significant first", [(bmm, "tensor_mle", _tensor_mle_lsb)]),
    ("eq(rho, h) weight dropped", [(bmm, "tensor_mle", _tensor_mle_no_head_weight)]),
]


def test_unmutated_oracle_passes_the_pins():
    assert _pins_hold()


@pytest.mark.parametrize("name,patches", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, patches, monkeypatch):
    for mod, attr, fn in patches:
        monkeypatch.setattr(mod, attr, fn)
    assert not _pins_hold(), f"pins did not catch: {name}"
