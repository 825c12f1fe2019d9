"""Pins of the lookup-argument oracle (oracle/lookup.py) against facts fixed outside it (no GPU).

Protocol 1 rests on the rational-function identity of eq. (rational-function)
and the sum of eq. (lookup-sumcheck).  The pins:
  * the multiplicities make sum 1/(b + s_i) = sum m_j/(b + t_j) hold exactly
    over the rationals (Python fractions) at several integers b, and fail to
    when one entry is moved;
  * the field form sum_i A_i = sum_j m_j B_j holds at the oracle's beta;
  * perfect completeness with every final value checked by direct MLE
    evaluation; every single-element tamper rejected; a value outside the
    table refused; wrong multiplicities refused by the sum;
  * each round polynomial has degree 3: the sum at X = 4 computed from the
    definition equals the cubic extrapolation;
  * with D = N the high part is empty; padding keeps S inside T;
  * the refined sum equals alpha + alpha^2 with the N/D factor and not
    without it; planted mistakes (gamma missing from the table, a swapped
    fold) are caught.
"""
import random
from fractions import Fraction

import pytest

import oracle.lookup as lk
import workloads
from oracle import P, enc, inv
from oracle.mle import eq_table
from oracle.zkmat import FalseStatement, Reject

CASES = [
    dict(seed=1, D=20, N=8, t0=-3, two_col=True),
    dict(seed=2, D=8, N=8, t0=5, two_col=False),
    dict(seed=3, D=64, N=4, t0=0, two_col=False),
    dict(seed=4, D=3, N=16, t0=-100, two_col=True),
    dict(seed=5, D=37, N=2, t0=7, two_col=False),
    dict(seed=6, D=1, N=1, t0=2, two_col=False),
]


def _case(i):
    c = dict(CASES[i])
    return workloads.tiny_lookup(c["seed"], c["D"], c["N"], c["t0"], c["two_col"])


def _wit(c):
    return (c.x.tolist(), c.y.tolist() if c.y is not None else None, c.tb.tolist() if c.tb is not None else None)


@pytest.mark.parametrize("i", range(len(CASES)))
def test_complete_with_witness(i):
    c = _case(i)
    proof, state, det = lk.prove_case(c, 9)
    assert len(proof) == lk.proof_len(len(c.x), c.N)
    res = lk.verify(proof, len(c.x), c.N, c.t0, c.y is not None, 9, c.lid, witness=_wit(c))
    assert res["state"] == state


def test_multiplicities_satisfy_the_rational_identity_over_q():
    c = workloads.tiny_lookup(11, 50, 16, t0=-8)
    m = lk.multiplicities(c.x.tolist(), None, c.t0, None, c.N)
    assert sum(m) == 50
    for b in (17, 1000, -1001, 12345):
        lhs = sum(Fraction(1, b + int(s)) for s in c.x)
        rhs = sum(Fraction(m[j], b + c.t0 + j) for j in range(c.N))
        assert lhs == rhs
    # one entry moved to another table value breaks it
    m2 = list(m)
    j = next(k for k in range(c.N) if m2[k] > 0)
    m2[j] -= 1
    m2[(j + 1) % c.N] += 1
    b = 1000
    assert sum(Fraction(1, b + int(s)) for s in c.x) != sum(Fraction(m2[k], b + c.t0 + k) for k in range(c.N))


def test_field_form_of_the_identity_at_beta():
    c = _case(0)
    _, _, det = lk.prove_case(c, 3)
    beta, gamma, m = det["beta"], det["gamma"], det["m"]
    S = [(int(x) + gamma * int(y)) % P for x, y in zip(c.x, c.y)] + \
        [(c.t0 + gamma * int(c.tb[0])) % P] * (det["Dp"] - len(c.x))
    T = [(c.t0 + j + gamma * int(c.tb[j])) % P for j in range(c.N)]
    assert sum(inv(beta + s) for s in S) % P == sum(m[j] * inv(beta + T[j]) for j in range(c.N)) % P


def test_value_outside_the_table_is_refused():
    c = _case(1)
    x = c.x.copy()
    x[3] = c.t0 + c.N        # one past the end
    with pytest.raises(FalseStatement):
        lk.prove(x.tolist(), None, c.t0, None, c.N, 1, 0)
    c = _case(0)
    y = c.y.copy()
    y[0] += 1                # input in range, output not the table's
    with pytest.raises(FalseStatement):
        lk.prove(c.x.tolist(), y.tolist(), c.t0, c.tb.tolist(), c.N, 1, 0)


def test_wrong_multiplicities_are_refused_by_the_sum():
    c = _case(2)
    m = lk.multiplicities(c.x.tolist(), None, c.t0, None, c.N)
    m[0] += 1
    m[1] -= 1
    with pytest.raises(FalseStatement):
        lk.prove(c.x.tolist(), None, c.t0, None, c.N, 1, 0, m_override=m)


@pytest.mark.parametrize("i", [0, 2, 4])
def test_every_single_element_tamper_is_rejected(i):
    c = _case(i)
    proof, _, _ = lk.prove_case(c, 21)
    for pos in range(0, len(proof), 32):
        x = int.from_bytes(proof[pos:pos + 32], "little")
        bad = proof[:pos] + enc((x + 1) % P) + proof[pos + 32:]
        with pytest.raises(Reject):
            lk.verify(bad, len(c.x), c.N, c.t0, c.y is not None, 21, c.lid, witness=_wit(c))
    with pytest.raises(Reject):
        lk.verify(proof, len(c.x), c.N, c.t0, c.y is not None, 22, c.lid)


@pytest.mark.parametrize("i", [0, 3, 4])
def test_round_polynomials_have_degree_three(i):
    # rebuild the summand's tables from the definitions, fold them with the
    # proof's challenges, and compare the round sum at X = 4 with the cubic
    # through the sent values
    c = _case(i)
    _, _, det = lk.prove_case(c, 13)
    Dp, N, nH = det["Dp"], c.N, det["nH"]
    beta, gamma, alpha, u, m = det["beta"], det["gamma"], det["alpha"], det["u"], det["m"]
    two = c.y is not None
    xs = [int(v) for v in c.x] + [c.t0] * (Dp - len(c.x))
    ys = ([int(v) for v in c.y] + [int(c.tb[0])] * (Dp - len(c.x))) if two else [0] * Dp
    tbv = [int(v) for v in c.tb] if two else [0] * N
    Sb = [(xs[i] + gamma * ys[i] + beta) % P for i in range(Dp)]
    Tb = [(c.t0 + j + gamma * tbv[j] + beta) % P for j in range(N)]
    A = [inv(s) for s in Sb]
    E, EL = eq_table(u), eq_table(u[nH:])
    c2 = N * inv(Dp) % P
    c1 = c2 * alpha * alpha % P
    tabs = dict(E=E, A=A, S=Sb, B=[inv(Tb[i % N]) for i in range(Dp)], L=[EL[i % N] for i in range(Dp)],
                T=[Tb[i % N] for i in range(Dp)], M=[m[i % N] for i in range(Dp)])
    for g, r in zip(det["rounds"], det["r"]):
        h = len(tabs["A"]) // 2
        at = {k: [(v[t] + 4 * (v[t + h] - v[t])) % P for t in range(h)] for k, v in tabs.items()}
        s4 = sum(alpha * at["E"][t] * at["A"][t] * at["S"][t] + at["A"][t] + c1 * at["B"][t] * at["L"][t] * at["T"][t]
                 - c2 * at["B"][t] * at["M"][t] for t in range(h)) % P
        from oracle.bmm import lagrange_eval
        assert s4 == lagrange_eval(g, 4)
        tabs = {k: [(v[t] + r * (v[t + h] - v[t])) % P for t in range(h)] for k, v in tabs.items()}


def test_padding_keeps_entries_in_the_table():
    c = _case(4)       # D = 37 -> 64
    _, _, det = lk.prove_case(c, 2)
    assert det["Dp"] == 64
    assert sum(det["m"]) == 64 and det["m"][0] >= 64 - 37


# ----------------------------------------------------- planted mistakes --
def _pins_hold() -> bool:
    try:
        for i in (0, 2, 4):
            c = _case(i)
            proof, _, _ = lk.prove_case(c, 7)
            lk.verify(proof, len(c.x), c.N, c.t0, c.y is not None, 7, c.lid, witness=_wit(c))
    except (Reject, FalseStatement, AssertionError, ValueError, IndexError, ZeroDivisionError):
        return False
    return True


_orig_setup = lk._setup
_orig_line = lk._line


def _setup_table_without_gamma(*args):
    st = _orig_setup(*args)
    xs, ys, t0, tb, N = args[0], args[1], args[2], args[3], args[4]
    if tb is not None:
        st["T"] = [(t0 + j) % P for j in range(N)]
    return st


def _line_swapped(x, h, X):
    return (x[h:2 * h] + X * (x[:h] - x[h:2 * h])) % P


MUTATIONS = [
    ("table built without gamma", [(lk, "_setup", _setup_table_without_gamma)]),
    ("fold weights swapped", [(lk, "_line", _line_swapped)]),
]


def test_unmutated_oracle_passes_the_pins():
    assert _pins_hold()


@pytest.mark.parametrize("name,patches", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, patches, monkeypatch):
    for mod, attr, fn in patches:
        monkeypatch.setattr(mod, attr, fn)
    assert not _pins_hold(), f"pins did not catch: {name}"


def test_dropping_the_n_over_d_factor_breaks_the_sum():
    c = _case(2)
    st = lk._setup(c.x.tolist(), None, c.t0, None, c.N, 1, 0)
    m = lk.multiplicities(st["xs"], None, c.t0, None, c.N)
    beta, alpha, u, Dp, N, nH = st["beta"], st["alpha"], st["u"], st["Dp"], c.N, st["nH"]
    E, EL = eq_table(u), eq_table(u[nH:])
    A = [inv(s + beta) for s in st["S"]]
    B = [inv(t + beta) for t in st["T"]]
    Tb = [(t + beta) % P for t in st["T"]]
    full = sum(alpha * E[i] * A[i] * (st["S"][i] + beta) + A[i] for i in range(Dp))
    low = sum(alpha * alpha * B[i % N] * EL[i % N] * Tb[i % N] - B[i % N] * m[i % N] for i in range(Dp))
    with_factor = (full + N * inv(Dp) * low) % P
    without = (full + low) % P
    assert with_factor == (alpha + alpha * alpha) % P
    assert without != (alpha + alpha * alpha) % P
