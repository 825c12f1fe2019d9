"""Host-side checks of the batched-product ABI (no GPU).

The library's host verifier of the per-head batched sumcheck (C++
transcript, cubic and quadratic interpolation, 3-D MLE witness evaluation)
must accept every proof the oracle wrote for the stored cases, return the
oracle's challenges, and reject every single-element tamper; the size
queries must agree with the oracle's proof length and plan without a GPU.
"""
import json
import os

import pytest

import oracle.bmm as obmm
import workloads
from paper_2508_21393_amd import binding as B
from bmm_util import bmm_args

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden", "bmm.json")


def _lib_or_skip():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libverilora.so not built")
    return B.lib()


def _tiny_cases():
    spec = json.load(open(GOLD))
    out = []
    for k, (seed, H, d0, d1, d2, kw) in enumerate(spec["tiny_spec"]):
        hb = workloads.tiny_head_batch(seed, H, d0, d1, d2, name=f"bmm{k}", **kw)
        hb.group_id = k
        out.append((hb, bytes.fromhex(spec["tiny"][k]["proof_hex"]), spec["seed"]))
    small = workloads.attention_layer(**spec["attn_small_spec"])
    for hb, e in zip(small, spec["attn_small"]):
        out.append((hb, bytes.fromhex(e["proof_hex"]), spec["seed"]))
    return out


def test_sizes_match_the_oracle():
    _lib_or_skip()
    for hb, proof, _ in _tiny_cases():
        H, d0, d1, d2 = hb.dims
        assert B.bmm_proof_size(bmm_args(hb, "none")) == obmm.proof_len(H, d1) == len(proof)


def test_workspace_size_plans_on_the_host():
    _lib_or_skip()
    cases = [hb for hb, _, _ in _tiny_cases()]
    one = B.bmm_workspace_size([bmm_args(cases[0], "none")])
    both = B.bmm_workspace_size([bmm_args(hb, "none") for hb in cases])
    assert 0 < one < both


@pytest.mark.parametrize("i", range(18))
def test_host_verifier_accepts_oracle_proofs(i):
    _lib_or_skip()
    cases = _tiny_cases()
    if i >= len(cases):
        pytest.skip("no such case")
    hb, proof, seed = cases[i]
    ok, fr, red = B.bmm_verify(proof, bmm_args(hb, "host"), seed)
    assert ok, B.last_error()
    det = obmm.verify(proof, *hb.dims, seed, hb.group_id)
    assert red[0] == det["c"]
    nh = len(det["rho"])
    assert red[1:1 + nh] == det["rho"]
    tail = red[1 + nh + len(det["u"]) + len(det["v"]):]
    assert tail[:-2] == det["r"] and tail[-2:] == [det["a_final"], det["b_final"]]


@pytest.mark.parametrize("i", [1, 4, 7, 9])
def test_host_verifier_rejects_every_single_element_tamper(i):
    _lib_or_skip()
    hb, proof, seed = _tiny_cases()[i]
    args = bmm_args(hb, "host")
    for pos in range(0, len(proof), 32):
        x = int.from_bytes(proof[pos:pos + 32], "little")
        bad = proof[:pos] + ((x + 1) % oracle_p()).to_bytes(32, "little") + proof[pos + 32:]
        ok, _, _ = B.bmm_verify(bad, args, seed)
        assert not ok, pos
    ok, _, _ = B.bmm_verify(proof, bmm_args(hb, "host"), seed + 1)
    assert not ok


def oracle_p():
    from oracle import P
    return P


def test_host_verifier_rejects_a_wrong_witness():
    _lib_or_skip()
    hb, proof, seed = _tiny_cases()[1]
    A = hb.A.base.copy()
    A.reshape(-1)[0] += 1
    bad = workloads.HeadBatch(hb.name, workloads.HeadView(A, hb.A.H, hb.A.rows, hb.A.cols, hb.A.head_stride, hb.A.ld),
                              hb.B, hb.C, hb.transA, hb.transB, hb.group_id)
    ok, _, _ = B.bmm_verify(proof, bmm_args(bad, "host"), seed)
    assert not ok
    ok, _, _ = B.bmm_verify(proof, bmm_args(hb, "none"), seed)   # shape only: the sumcheck holds
    assert ok


def test_prove_refuses_bad_shapes_before_device_work():
    _lib_or_skip()
    hb = _tiny_cases()[1][0]
    import ctypes
    a = bmm_args(hb, "none")
    a.struct.lda = 0
    buf = ctypes.create_string_buffer(1 << 16)
    offs = (ctypes.c_uint64 * 2)()
    st = B.lib().vl_bmm_prove(ctypes.byref(a.struct), 1, 1, 256, 1 << 20, ctypes.addressof(buf), 1 << 16, offs,
                              None, None)
    assert st == B.VL_ERR_SHAPE
    a = bmm_args(hb, "none")   # null tensors
    st = B.lib().vl_bmm_prove(ctypes.byref(a.struct), 1, 1, 256, 1 << 20, ctypes.addressof(buf), 1 << 16, offs,
                              None, None)
    assert st == B.VL_ERR_INVALID_ARG
    a = bmm_args(hb, "none")
    a.struct.H = 0
    assert B.bmm_proof_size(a) == 0
