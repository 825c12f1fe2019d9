"""Pins of the layer chain oracle (oracle/chain.py) against facts fixed outside it (no GPU).

The chain composes zkMat steps (Sec. IV-B) and the update check of
eq. (grad_update_ab).  Its pins: completeness with every final and open
claim evaluated by the definition of eq. (MLE); rejection of every
single-element tamper; refusal of false statements; the algebraic identity
each reduction rests on, by brute force; the reduced value against direct
evaluation; the degree of the reduction's round polynomials by brute-force
extrapolation; the linearity that lets the update be checked at one point.
"""
import random

import numpy as np
import pytest

import oracle
import workloads
from oracle import P, eq_table, matrix_mle
from oracle.mle import eq_basis, bits_msb_first, num_vars
from oracle.chain import (chain_prove, chain_verify, chain_proof_len, reduce_prove, reduce_verify, TENSORS)
from oracle.transcript import Transcript
from oracle.zkmat import FalseStatement, Reject, interpolate_quadratic

SHAPES = [(8, 12, 10, 3), (4, 4, 4, 2), (5, 7, 9, 1), (1, 3, 2, 2), (16, 8, 32, 4), (3, 1, 5, 1)]


def _rnd(rng, n):
    return [rng.randrange(P) for _ in range(n)]


@pytest.mark.parametrize("dims", SHAPES)
def test_chain_complete_with_witness(dims):
    w = workloads.tiny_layer(sum(dims), *dims)
    proof, state, det = chain_prove(w, 9)
    assert len(proof) == chain_proof_len(dims)
    res = chain_verify(proof, dims, 9, w.F, w.eta, witness=w)
    assert res["state"] == state
    assert set(res["reduced"]) == set(TENSORS)


def test_chain_final_claims_are_the_tensors_mles():
    # every claim the verifier ends with equals the tensor's multilinear
    # extension at that point, evaluated here by the definition of eq. (MLE)
    # with an explicit double sum (not matrix_mle)
    dims = (4, 6, 5, 2)
    w = workloads.tiny_layer(3, *dims)
    proof, _, _ = chain_prove(w, 4)
    res = chain_verify(proof, dims, 4, w.F, w.eta)

    def direct(M, x, y):
        tot = 0
        for i in range(M.shape[0]):
            for j in range(M.shape[1]):
                tot += int(M[i, j]) * eq_basis(x, bits_msb_first(i, len(x))) * eq_basis(y, bits_msb_first(j, len(y)))
        return tot % P

    for name, red in res["reduced"].items():
        assert direct(getattr(w, name), red["r"], red["s"]) == red["value"], name
    for name, (x, y, v) in res["open"].items():
        assert direct(getattr(w, name), x, y) == v, name


def test_every_single_element_tamper_is_rejected():
    dims = (4, 6, 5, 2)
    w = workloads.tiny_layer(5, *dims)
    proof, _, _ = chain_prove(w, 11)
    for i in range(len(proof) // 32):
        x = int.from_bytes(proof[32 * i:32 * i + 32], "little")
        bad = proof[:32 * i] + ((x + 1) % P).to_bytes(32, "little") + proof[32 * i + 32:]
        with pytest.raises(Reject):
            chain_verify(bad, dims, 11, w.F, w.eta)
    with pytest.raises(Reject):
        chain_verify(proof, dims, 12, w.F, w.eta)          # another seed
    with pytest.raises(Reject):
        chain_verify(proof, dims, 11, w.F, w.eta + 1)      # another learning rate
    with pytest.raises(Reject):
        chain_verify(proof[:-32], dims, 11, w.F, w.eta)


def test_wrong_witness_tensor_is_rejected():
    dims = (4, 6, 5, 2)
    w = workloads.tiny_layer(6, *dims)
    proof, _, _ = chain_prove(w, 2)
    for name in ("X", "W", "A", "B", "dY", "H", "G", "UA", "UB", "Y", "dX", "C2", "C4"):
        bad = workloads.LayerWitness(**{k: getattr(w, k) for k in w.__dataclass_fields__})
        M = getattr(bad, name).copy()
        M.flat[-1] += 1
        setattr(bad, name, M)
        with pytest.raises(Reject):
            chain_verify(proof, dims, 2, w.F, w.eta, witness=bad)


@pytest.mark.parametrize("name", ["UA", "UB", "dA", "dB", "Y", "dX", "C2", "C4"])
def test_false_statements_are_refused(name):
    dims = (4, 6, 5, 2)
    w = workloads.tiny_layer(7, *dims)
    bad = workloads.LayerWitness(**{k: getattr(w, k) for k in w.__dataclass_fields__})
    M = getattr(bad, name).copy()
    M[0, 0] += 1
    setattr(bad, name, M)
    if name in ("dA", "dB"):
        # keep the update relation true for the wrong gradient: then its
        # product sumcheck must refuse
        U = "UA" if name == "dA" else "UB"
        base = bad.A if name == "dA" else bad.B
        setattr(bad, U, (base.astype(np.int64) << bad.F) - bad.eta * M)
    with pytest.raises(FalseStatement):
        chain_prove(bad, 1)


def test_update_relation_is_linear_in_the_mles():
    # UA = 2^F A - eta dA entrywise makes UA~ = 2^F A~ - eta dA~ at any point
    # (the MLE is linear in the table), the fact the stage-1 check rests on
    w = workloads.tiny_layer(8, 6, 9, 7, 3)
    assert np.array_equal(w.UA, (w.A.astype(np.int64) << w.F) - w.eta * w.dA)
    rng = random.Random(1)
    for _ in range(3):
        x, y = _rnd(rng, num_vars(9)), _rnd(rng, num_vars(3))
        assert matrix_mle(w.UA, x, y) == ((1 << w.F) * matrix_mle(w.A, x, y) - w.eta * matrix_mle(w.dA, x, y)) % P


def _claims(rng, M, K):
    nR, nC = num_vars(M.shape[0]), num_vars(M.shape[1])
    out = []
    for _ in range(K):
        x, y = _rnd(rng, nR), _rnd(rng, nC)
        out.append((x, y, matrix_mle(M, x, y)))
    return out


@pytest.mark.parametrize("shape,K", [((5, 7), 3), ((8, 8), 2), ((1, 6), 2), ((6, 1), 3), ((2, 2), 1)])
def test_reduction_identity_by_brute_force(shape, K):
    # sum_k rho_k v_k = sum_{i,j} M[i,j] sum_k rho_k eq(x_k, i) eq(y_k, j),
    # summed entry by entry
    rng = random.Random(shape[0] * 31 + K)
    M = np.array([[rng.randrange(-99, 99) for _ in range(shape[1])] for _ in range(shape[0])], dtype=np.int64)
    claims = _claims(rng, M, K)
    rho = _rnd(rng, K)
    ex = [eq_table(x) for x, _, _ in claims]
    ey = [eq_table(y) for _, y, _ in claims]
    rhs = 0
    for i in range(shape[0]):
        for j in range(shape[1]):
            rhs += int(M[i, j]) * sum(rho[k] * ex[k][i] * ey[k][j] for k in range(K))
    assert rhs % P == sum(rho[k] * claims[k][2] for k in range(K)) % P


@pytest.mark.parametrize("shape,K", [((5, 7), 3), ((8, 8), 2), ((1, 6), 2), ((6, 1), 3), ((3, 3), 1)])
def test_reduction_complete_and_value_is_the_mle(shape, K):
    rng = random.Random(shape[1] * 17 + K)
    M = np.array([[rng.randrange(-(1 << 15), 1 << 15) for _ in range(shape[1])] for _ in range(shape[0])],
                 dtype=np.int64)
    claims = _claims(rng, M, K)
    tr = Transcript.from_state(b"\x07" * 32)
    proof, det = reduce_prove(tr, M, claims)
    tv = Transcript.from_state(b"\x07" * 32)
    res = reduce_verify(tv, shape, claims, proof)
    assert tv.state == tr.state
    assert res["value"] == matrix_mle(M, res["r"], res["s"]) == det["value"]
    # t_k(r) sent after the row rounds are M~(r, y_k)
    assert det["t"] == [matrix_mle(M, det["r"], y) for _, y, _ in claims]


def test_reduction_rejects_a_false_claim_value():
    rng = random.Random(4)
    M = np.array([[rng.randrange(-50, 50) for _ in range(6)] for _ in range(5)], dtype=np.int64)
    claims = _claims(rng, M, 3)
    bad = list(claims)
    x, y, v = bad[1]
    bad[1] = (x, y, (v + 1) % P)
    proof, _ = reduce_prove(Transcript.from_state(b"\x01" * 32), M, bad)
    with pytest.raises(Reject):
        reduce_verify(Transcript.from_state(b"\x01" * 32), M.shape, bad, proof)


def test_reduction_row_rounds_have_degree_two():
    # the first row round's g(3), computed from the full tables by the
    # definition (each table extended linearly in the bound variable), equals
    # the quadratic through g(0), g(1), g(2)
    rng = random.Random(9)
    M = np.array([[rng.randrange(-70, 70) for _ in range(4)] for _ in range(8)], dtype=np.int64)
    claims = _claims(rng, M, 3)
    tr = Transcript.from_state(b"\x02" * 32)
    proof, det = reduce_prove(tr, M, claims)
    g0, g1, g2 = (int.from_bytes(proof[32 * k:32 * k + 32], "little") for k in range(3))
    from oracle.mle import partial_eval_cols
    h = 4
    g3 = 0
    for k, (x, y, _) in enumerate(claims):
        e, t = eq_table(x), partial_eval_cols(M, y)
        for i in range(h):
            e3 = e[i] + 3 * (e[i + h] - e[i])
            t3 = t[i] + 3 * (t[i + h] - t[i])
            g3 += det["rho"][k] * e3 * t3
    assert g3 % P == interpolate_quadratic(g0, g1, g2, 3)


# ------------------------------------------------------- planted mistakes ---
import oracle.chain as ch  # noqa: E402


def _chain_pins_hold() -> bool:
    try:
        for dims in ((4, 6, 5, 2), (3, 5, 4, 1)):
            w = workloads.tiny_layer(sum(dims) + 1, *dims)
            proof, _, _ = ch.chain_prove(w, 3)
            ch.chain_verify(proof, dims, 3, w.F, w.eta, witness=w)
        rng = random.Random(2)
        M = np.array([[rng.randrange(-9, 9) for _ in range(5)] for _ in range(6)], dtype=np.int64)
        claims = _claims(rng, M, 3)
        proof, det = ch.reduce_prove(Transcript.from_state(b"\x05" * 32), M, claims)
        res = ch.reduce_verify(Transcript.from_state(b"\x05" * 32), M.shape, claims, proof)
        if res["value"] != matrix_mle(M, res["r"], res["s"]):
            return False
    except (Reject, FalseStatement, AssertionError, ValueError, IndexError):
        return False
    return True


def _claims_untransposed(pts, nv, details, upd):
    c = _orig_collect(pts, nv, details, upd)
    x, y, v = c["X"][2]
    c["X"][2] = (y, x, v)               # X^T's claim read as if X were not transposed
    return c


def _reduce_prove_rho_for_sigma(tr, M, claims):
    # phase 2 built with the row combination's coefficients
    K = len(claims)
    saved = ch._squeeze

    def sq(t, label, n):
        return saved(t, b"rho" if label == b"sigma" else label, n)
    ch._squeeze = sq
    try:
        return _orig_reduce(tr, M, claims)
    finally:
        ch._squeeze = saved


def _eq_table_lsb(x):
    n = len(x)
    return [eq_basis(x, [(i >> j) & 1 for j in range(n)]) for i in range(1 << n)]


_orig_collect = ch.collect_claims
_orig_reduce = ch.reduce_prove

MUTATIONS = [
    ("collect_claims", _claims_untransposed),
    ("reduce_prove", _reduce_prove_rho_for_sigma),
    ("eq_table", _eq_table_lsb),
]


def test_chain_pins_hold_unmutated():
    assert _chain_pins_hold()


@pytest.mark.parametrize("name,bad", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_chain_mistake_is_caught(monkeypatch, name, bad):
    monkeypatch.setattr(ch, name, bad)
    assert not _chain_pins_hold()
