"""Per-head batched products on the GPU against the oracle (needs a gfx950 GPU).

vl_bmm_prove must write exactly the oracle's bytes (oracle/bmm.py): the tiny
cases (heads side by side in columns or stacked, transposed views, padding
heads, ragged dimensions, tables large enough for the GPU-wide rounds, one
head) and a small attention layer against the full proofs in
tests/golden/bmm.json, and the 7B-class attention layer (T = 2048, 32 heads
of 128: S = Q K^T, O = P V, dP = dO V^T, dV = P^T dO, dQ = dS K,
dK = dS^T Q) against its stored digests.  False statements are refused
whether the guard fails in a GPU-wide round or in the one-workgroup rounds.
"""
import sys

import numpy as np
import pytest

import workloads
from bmm_util import bmm_args
from gpu_util import golden, sha, to_dev

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_21393_amd import binding
    binding.lib()
    return binding


def _tiny():
    spec = golden("bmm")
    out = []
    for k, (seed, H, d0, d1, d2, kw) in enumerate(spec["tiny_spec"]):
        hb = workloads.tiny_head_batch(seed, H, d0, d1, d2, name=f"bmm{k}", **kw)
        hb.group_id = k
        out.append((hb, spec["tiny"][k]))
    return out, spec["seed"]


def test_tiny_cases_one_call_match_oracle_bytes(B):
    cases, seed = _tiny()
    _say(f"bmm tiny: {len(cases)} products in one call")
    args = [bmm_args(hb, "device", to_dev) for hb, _ in cases]
    proofs, digs = B.bmm_prove(args, seed)
    for (hb, rec), p, d in zip(cases, proofs, digs):
        assert p.hex() == rec["proof_hex"], rec["name"]
        assert d.hex() == rec["state"], rec["name"]


def test_tiny_cases_one_by_one_match_oracle_bytes(B):
    cases, seed = _tiny()
    for hb, rec in cases:
        _say(f"bmm tiny {rec['name']} {hb.dims}")
        proofs, digs = B.bmm_prove([bmm_args(hb, "device", to_dev)], seed)
        assert proofs[0].hex() == rec["proof_hex"], rec["name"]
        assert digs[0].hex() == rec["state"], rec["name"]


def test_small_attention_layer_matches_oracle_bytes(B):
    spec = golden("bmm")
    layer = workloads.attention_layer(**spec["attn_small_spec"])
    _say("bmm small attention layer")
    proofs, digs = B.bmm_prove([bmm_args(hb, "device", to_dev) for hb in layer], spec["seed"])
    for hb, rec, p, d in zip(layer, spec["attn_small"], proofs, digs):
        assert p.hex() == rec["proof_hex"], rec["name"]
        assert d.hex() == rec["state"], rec["name"]
        ok, fr, _ = B.bmm_verify(p, bmm_args(hb, "none"), spec["seed"])
        assert ok, (rec["name"], fr, B.last_error())


def test_full_size_attention_layer_matches_oracle(B):
    spec = golden("bmm")
    _say("bmm 7B-class attention layer: generating")
    layer = workloads.attention_layer(**spec["attn_full_spec"], device="cuda")
    args = [bmm_args(hb, "device", to_dev) for hb in layer]
    _say("bmm 7B-class attention layer: proving")
    proofs, digs = B.bmm_prove(args, spec["seed"])
    for hb, rec, p, d in zip(layer, spec["attn_full"], proofs, digs):
        assert list(hb.dims) == rec["dims"]
        assert len(p) == rec["proof_len"]
        assert sha(p) == rec["proof_sha256"], rec["name"]
        assert d.hex() == rec["state"], rec["name"]
        ok, fr, _ = B.bmm_verify(p, bmm_args(hb, "none"), spec["seed"])
        assert ok, (rec["name"], fr)
    _say("bmm 7B-class attention layer: second call, same tensors")
    proofs2, _ = B.bmm_prove(args, spec["seed"])
    assert proofs2 == proofs


@pytest.mark.parametrize("k", [1, 10, 11])
def test_false_statement_refused(B, k):
    # case 1: every round in one workgroup; cases 10, 11: the guard is
    # checked in the first GPU-wide round
    cases, seed = _tiny()
    hb, _ = cases[k]
    C = hb.C.base.copy()
    C.reshape(-1)[hb.C.head_stride * (hb.C.H - 1)] += 1    # first entry of the last head
    bad = workloads.HeadBatch(hb.name, hb.A, hb.B,
                              workloads.HeadView(C, hb.C.H, hb.C.rows, hb.C.cols, hb.C.head_stride, hb.C.ld),
                              hb.transA, hb.transB, hb.group_id)
    _say(f"bmm false statement in case {k}")
    with pytest.raises(B.VLError) as e:
        B.bmm_prove([bmm_args(bad, "device", to_dev)], seed)
    assert e.value.status == B.VL_ERR_FALSE_STATEMENT


def test_range_error_on_oversized_claim_entry(B):
    cases, seed = _tiny()
    hb, _ = cases[5]
    C = hb.C.base.copy()
    C.reshape(-1)[0] = 1 << 50
    bad = workloads.HeadBatch(hb.name, hb.A, hb.B,
                              workloads.HeadView(C, hb.C.H, hb.C.rows, hb.C.cols, hb.C.head_stride, hb.C.ld),
                              hb.transA, hb.transB, hb.group_id)
    _say("bmm range error")
    with pytest.raises(B.VLError) as e:
        B.bmm_prove([bmm_args(bad, "device", to_dev)], seed)
    assert e.value.status == B.VL_ERR_RANGE
