"""Host verifier with bind digests (CPU only; no device work).

Proofs bound to a commitment digest come from the oracle; the library's
verifier (vl_verify_transcript) must accept them under the same digest, give
the oracle's reduced claims, reject them under another digest or none, and
run without a witness, the reduced claims then checked by Hyrax openings
(vl_hyrax_verify_open) against the commitments the digest was made from
(Sec. II-C after II-A).
"""
import hashlib
import os

import numpy as np
import pytest

import workloads
from oracle import hyrax
from oracle.zkmat import prove_group, verify_group

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    from paper_2508_21393_amd import binding
    if not os.path.exists(os.path.join(ROOT, "paper_2508_21393_amd", "libverilora.so")):
        pytest.skip("library not built")
    binding.lib()
    return binding


def _host_group(B, g, bind=None):
    return B.GroupArgs(g.group_id, [(p.A, p.B, p.transA, p.transB) for p in g.products], g.C, bind=bind)


def test_bound_proofs_verify_under_their_digest(B):
    g = workloads.tiny_random_group(14, [(6, 10, 5), (6, 3, 5)], trans=(True, False))
    prods = [(p.opA(), p.opB()) for p in g.products]
    d = hashlib.sha256(b"commitments").digest()
    proof, _, _ = prove_group(prods, g.C, 21, 0, bind=d)
    ok, fr, red = B.verify_transcript(proof, _host_group(B, g, d), 21)
    assert ok and fr == -1, B.last_error()
    res = verify_group(proof, g.shapes, 21, 0, bind=d)
    expect = [res["c"]] + res["u"] + res["v"]
    for rvec, (af, bf) in zip(res["r"], res["finals"]):
        expect += rvec + [af, bf]
    assert red == expect
    for other in (None, hashlib.sha256(b"other").digest()):
        assert not B.verify_transcript(proof, _host_group(B, g, other), 21)[0]
    # the unbound proof is not accepted under the digest either
    plain, _, _ = prove_group(prods, g.C, 21, 0)
    assert not B.verify_transcript(plain, _host_group(B, g, d), 21)[0]


def test_bind_length_is_checked(B):
    g = workloads.tiny_random_group(3, [(2, 2, 2)])
    for bad in (b"", bytes(31), bytes(33)):
        with pytest.raises(ValueError):
            _host_group(B, g, bad)


def test_commit_prove_open_on_the_host(B):
    # commitments to A, B and C (oracle Hyrax), a proof bound to their
    # digest, the library verifier without a witness, and the library's
    # opening verifier on each reduced claim
    rng = np.random.default_rng(40)
    A = rng.integers(-300, 300, size=(4, 8)).astype(np.int16)
    Bm = rng.integers(-300, 300, size=(8, 2)).astype(np.int16)
    C = A.astype(np.int64) @ Bm.astype(np.int64)
    gens = hyrax.generators(8)
    cA, cB, cC = hyrax.commit(A, gens), hyrax.commit(Bm, gens[:2]), hyrax.commit(C, gens[:2])
    enc = [b"".join(hyrax.encode(P) for P in cl) for cl in (cA, cB, cC)]
    d = hashlib.sha256(b"".join(enc)).digest()
    proof, _, _ = prove_group([(A, Bm)], C, 2, 0, bind=d)

    ga = B.GroupArgs.shapes_only(0, [(4, 8, 2)], bind=d)
    ok, fr, red = B.verify_transcript(proof, ga, 2)
    assert ok, B.last_error()
    c, u, v, r, af, bf = red[0], red[1:3], red[3:4], red[4:7], red[7], red[8]

    def opened(commits, R, m, M, x, y):
        okk, val, msg = B.hyrax_verify_open(commits, R, m, x, y, hyrax.open_at(M, x))
        assert okk, msg
        return val

    assert opened(enc[0], 4, 8, A, u, r) == af
    assert opened(enc[1], 8, 2, Bm, r, v) == bf
    assert opened(enc[2], 4, 2, C, u, v) == c
    # an opening of another matrix fails against the commitment
    A2 = A.copy()
    A2[0, 0] += 1
    okk, _, _ = B.hyrax_verify_open(enc[0], 4, 8, u, r, hyrax.open_at(A2, u))
    assert not okk
