"""Host-side checks of the lookup ABI (no GPU).

The library's host verifier of the lookup sumcheck (C++ transcript, cubic
interpolation, the summand of eq. (lookup-sumcheck) at the final point, and
the multilinear extensions of the witness) must accept every proof the
oracle wrote for the stored cases, return the oracle's challenges, and
reject every single-element tamper; the size queries must agree with the
oracle's proof length and plan without a GPU.
"""
import ctypes
import json
import os

import pytest

import oracle.lookup as olk
import workloads
from oracle import P
from paper_2508_21393_amd import binding as B
from lookup_util import lookup_args

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden", "lookup.json")


def _lib_or_skip():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libverilora.so not built")
    return B.lib()


def _cases():
    spec = json.load(open(GOLD))
    out = []
    for k, (s, D, N, t0, two) in enumerate(spec["tiny_spec"]):
        out.append((workloads.tiny_lookup(s, D, N, t0, two, lid=k), bytes.fromhex(spec["tiny"][k]["proof_hex"])))
    for k, (kind, s, D) in enumerate(spec["mid_spec"]):
        lc = (workloads.lookup_range if kind == "range" else workloads.lookup_silu)(s, D, k)
        out.append((lc, bytes.fromhex(spec["mid"][k]["proof_hex"])))
    return out, spec["seed"]


def test_sizes_match_the_oracle():
    _lib_or_skip()
    cases, _ = _cases()
    for lc, proof in cases:
        assert B.lookup_proof_size(lookup_args(lc, "none")) == olk.proof_len(len(lc.x), lc.N) == len(proof)


def test_workspace_size_plans_on_the_host():
    _lib_or_skip()
    cases, _ = _cases()
    one = B.lookup_workspace_size([lookup_args(cases[0][0], "none")])
    all_ = B.lookup_workspace_size([lookup_args(lc, "none") for lc, _ in cases])
    assert 0 < one < all_


@pytest.mark.parametrize("i", range(11))
def test_host_verifier_accepts_oracle_proofs(i):
    _lib_or_skip()
    cases, seed = _cases()
    lc, proof = cases[i]
    ok, fr, red = B.lookup_verify(proof, lookup_args(lc, "host"), seed)
    assert ok, B.last_error()
    det = olk.verify(proof, len(lc.x), lc.N, lc.t0, lc.y is not None, seed, lc.lid)
    assert red[:3] == [det["gamma"], det["beta"], det["alpha"]]
    n = len(det["u"])
    assert red[3:3 + n] == det["u"] and red[3 + n:3 + 2 * n] == det["r"]
    assert red[3 + 2 * n:] == det["finals"]


@pytest.mark.parametrize("i", [0, 2, 6])
def test_host_verifier_rejects_every_single_element_tamper(i):
    _lib_or_skip()
    cases, seed = _cases()
    lc, proof = cases[i]
    args = lookup_args(lc, "host")
    for pos in range(0, len(proof), 32):
        x = int.from_bytes(proof[pos:pos + 32], "little")
        bad = proof[:pos] + ((x + 1) % P).to_bytes(32, "little") + proof[pos + 32:]
        ok, _, _ = B.lookup_verify(bad, args, seed)
        assert not ok, pos
    ok, _, _ = B.lookup_verify(proof, args, seed + 1)
    assert not ok


def test_host_verifier_rejects_a_wrong_witness():
    _lib_or_skip()
    cases, seed = _cases()
    lc, proof = cases[2]
    x = lc.x.copy()
    x[0] = lc.t0 + (int(x[0]) - lc.t0 + 1) % lc.N     # another row of the table
    bad = workloads.LookupCase(lc.name, x, lc.y, lc.t0, lc.tb, lc.N, lc.lid)
    ok, _, _ = B.lookup_verify(proof, lookup_args(bad, "host"), seed)
    assert not ok
    ok, _, _ = B.lookup_verify(proof, lookup_args(lc, "none"), seed)
    assert ok


def test_prove_refuses_bad_arguments_before_device_work():
    _lib_or_skip()
    cases, _ = _cases()
    lc = cases[0][0]
    buf = ctypes.create_string_buffer(1 << 16)
    offs = (ctypes.c_uint64 * 2)()
    a = lookup_args(lc, "none")
    a.struct.N = 12           # not a power of two
    st = B.lib().vl_lookup_prove(ctypes.byref(a.struct), 1, 1, 256, 1 << 20, ctypes.addressof(buf), 1 << 16, offs,
                                 None, None)
    assert st == B.VL_ERR_SHAPE
    a = lookup_args(lc, "none")   # null entries
    st = B.lib().vl_lookup_prove(ctypes.byref(a.struct), 1, 1, 256, 1 << 20, ctypes.addressof(buf), 1 << 16, offs,
                                 None, None)
    assert st == B.VL_ERR_INVALID_ARG
    a = lookup_args(lc, "none")
    a.struct.dtype = B.VL_I64
    assert B.lookup_proof_size(a) == 0
