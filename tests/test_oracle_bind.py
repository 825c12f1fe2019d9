"""Pins of the oracle's commitment binding (CPU only).

Sec. II-C has the verifier draw its random point only after the prover has
committed to the matrices (Sec. II-A).  A group's transcript takes an
optional 32-byte digest of the commitments ("bind") before u and v.  The
pins: no bind leaves every stored proof as it was; a bound proof verifies
only under its own digest; and the composed protocol (Hyrax row commitments,
bound sumcheck, openings of the reduced claims) accepts an honest prover and
rejects one that proves a true product of other matrices than those it
committed to, whichever opening it then sends.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from oracle import hyrax
from oracle.zkmat import Reject, challenges_uv, group_transcript, prove_group, verify_group

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _digest(*commit_lists) -> bytes:
    return hashlib.sha256(b"".join(hyrax.encode(P) for cl in commit_lists for P in cl)).digest()


def test_no_bind_keeps_the_stored_proofs():
    spec = json.load(open(os.path.join(GOLD, "tiny.json")))
    for k, (seed, dims, dt, trans, vb) in enumerate(spec["tiny_spec"][:4]):
        g = workloads.tiny_random_group(seed, [tuple(d) for d in dims], dtype=getattr(np, dt),
                                        trans=tuple(trans), value_bits=vb)
        prods = [(p.opA(), p.opB()) for p in g.products]
        proof, _, _ = prove_group(prods, g.C, spec["seed"], k, bind=None)
        assert proof.hex() == spec["groups"][k]["proof_hex"]


def test_bound_proof_verifies_only_under_its_digest():
    g = workloads.tiny_random_group(8, [(4, 8, 4), (4, 2, 4)])
    prods = [(p.opA(), p.opB()) for p in g.products]
    d1, d2 = hashlib.sha256(b"one").digest(), hashlib.sha256(b"two").digest()
    proof, _, _ = prove_group(prods, g.C, 5, 0, bind=d1)
    res = verify_group(proof, g.shapes, 5, 0, witness=(prods, g.C), bind=d1)
    assert res["c"] == oracle.matrix_mle(g.C, res["u"], res["v"])
    # another digest or none: other challenges, so the rounds no longer hold
    for other in (d2, None):
        with pytest.raises(Reject):
            verify_group(proof, g.shapes, 5, 0, bind=other)
    # the unbound proof differs from the bound one
    assert prove_group(prods, g.C, 5, 0)[0] != proof


def test_bind_moves_the_challenges():
    shapes = [(16, 8, 16)]
    points = set()
    for bind in (None, bytes(32), b"\x01" + bytes(31), hashlib.sha256(b"x").digest()):
        u, v = challenges_uv(group_transcript(3, 0, shapes, bind), shapes)
        points.add(tuple(u + v))
    assert len(points) == 4


def test_bind_must_be_32_bytes():
    for bad in (b"", bytes(31), bytes(33)):
        with pytest.raises(ValueError):
            group_transcript(1, 0, [(2, 2, 2)], bad)


def _committed_statement():
    rng = np.random.default_rng(12)
    A = rng.integers(-200, 200, size=(4, 8)).astype(np.int64)
    Bm = rng.integers(-200, 200, size=(8, 2)).astype(np.int64)
    C = A @ Bm
    gens = hyrax.generators(8)
    cA, cB, cC = hyrax.commit(A, gens), hyrax.commit(Bm, gens[:2]), hyrax.commit(C, gens[:2])
    return A, Bm, C, gens, (cA, cB, cC)


def _check_openings(res, commits, gens, opened):
    """The verifier's side: each reduced claim against an opening of its
    committed matrix (A at (u, r), B at (r, v), C at (u, v))."""
    cA, cB, cC = commits
    (A, Bm, C) = opened
    u, v, r = res["u"], res["v"], res["r"][0]
    af, bf = res["finals"][0]
    a = hyrax.verify_open(cA, gens, u, r, hyrax.open_at(A, u))
    b = hyrax.verify_open(cB, gens[:2], r, v, hyrax.open_at(Bm, r))
    c = hyrax.verify_open(cC, gens[:2], u, v, hyrax.open_at(C, u))
    return a == af and b == bf and c == res["c"]


def test_commit_then_prove_accepts_the_committed_statement():
    A, Bm, C, gens, commits = _committed_statement()
    bind = _digest(*commits)
    proof, _, _ = prove_group([(A, Bm)], C, 9, 0, bind=bind)
    res = verify_group(proof, [(4, 8, 2)], 9, 0, bind=bind)
    assert _check_openings(res, commits, gens, (A, Bm, C))


def test_commit_then_prove_rejects_a_substituted_statement():
    # the prover commits to (A, B, C), then proves the true product A' B = C'
    # of another A' under that commitment's digest: the sumcheck alone
    # passes, but an honest opening of A or C contradicts the proof's
    # claims, and an opening of A' or C' fails against the commitments
    A, Bm, C, gens, commits = _committed_statement()
    bind = _digest(*commits)
    A2 = A.copy()
    A2[1, 3] += 1
    C2 = A2 @ Bm
    proof, _, _ = prove_group([(A2, Bm)], C2, 9, 0, bind=bind)
    res = verify_group(proof, [(4, 8, 2)], 9, 0, bind=bind)
    assert not _check_openings(res, commits, gens, (A, Bm, C))
    with pytest.raises(ValueError):
        _check_openings(res, commits, gens, (A2, Bm, C2))
