"""Lookup arguments on the GPU against the oracle (needs a gfx950 GPU).

vl_lookup_prove must write exactly the oracle's bytes (oracle/lookup.py):
the tiny cases (one and two columns, tables of 1 to 2^14 rows, padding,
tables as large as S, GPU-wide rounds in the high and the low part) and a
range check of 2^16 activations and a SiLU input/output check of 2^18
against the full proofs in tests/golden/lookup.json, and the 7B-class cases
(2^23 activations, tables of 2^16 rows) against their stored digests.
Entries outside the table are refused.
"""
import sys

import pytest

import workloads
from gpu_util import golden, sha, to_dev
from lookup_util import lookup_args

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


def _case(kind, s, D, k):
    return (workloads.lookup_range if kind == "range" else workloads.lookup_silu)(s, D, k)


def _tiny():
    spec = golden("lookup")
    return [(workloads.tiny_lookup(s, D, N, t0, two, lid=k), spec["tiny"][k])
            for k, (s, D, N, t0, two) in enumerate(spec["tiny_spec"])], spec["seed"]


def test_tiny_cases_one_call_match_oracle_bytes(B):
    cases, seed = _tiny()
    _say(f"lookup tiny: {len(cases)} lookups in one call")
    proofs, digs = B.lookup_prove([lookup_args(lc, "device", to_dev) for lc, _ in cases], seed)
    for (lc, rec), p, d in zip(cases, proofs, digs):
        assert p.hex() == rec["proof_hex"], rec["name"]
        assert d.hex() == rec["state"], rec["name"]


def test_tiny_cases_one_by_one_match_oracle_bytes(B):
    cases, seed = _tiny()
    for lc, rec in cases:
        _say(f"lookup tiny {rec['name']}")
        proofs, digs = B.lookup_prove([lookup_args(lc, "device", to_dev)], seed)
        assert proofs[0].hex() == rec["proof_hex"], rec["name"]
        assert digs[0].hex() == rec["state"], rec["name"]


def test_mid_size_cases_match_oracle_bytes(B):
    spec = golden("lookup")
    for k, (kind, s, D) in enumerate(spec["mid_spec"]):
        lc = _case(kind, s, D, k)
        _say(f"lookup {lc.name}")
        proofs, digs = B.lookup_prove([lookup_args(lc, "device", to_dev)], spec["seed"])
        assert proofs[0].hex() == spec["mid"][k]["proof_hex"], lc.name
        assert digs[0].hex() == spec["mid"][k]["state"], lc.name


def test_full_size_cases_match_oracle_digests(B):
    spec = golden("lookup")
    if "full" not in spec:
        pytest.skip("the 7B-class lookup digests are not in tests/golden/lookup.json")
    cases = [_case(kind, s, D, k) for k, (kind, s, D) in enumerate(spec["full_spec"])]
    _say("lookup 7B-class cases: proving both in one call")
    args = [lookup_args(lc, "device", to_dev) for lc in cases]
    proofs, digs = B.lookup_prove(args, spec["seed"])
    for lc, rec, p, d in zip(cases, spec["full"], proofs, digs):
        assert len(p) == rec["proof_len"]
        assert sha(p) == rec["proof_sha256"], lc.name
        assert d.hex() == rec["state"], lc.name
        ok, fr, _ = B.lookup_verify(p, lookup_args(lc, "none"), spec["seed"])
        assert ok, (lc.name, fr)


@pytest.mark.parametrize("k", [1, 6, 8])
def test_entry_outside_the_table_is_refused(B, k):
    cases, seed = _tiny()
    lc, _ = cases[k]
    x = lc.x.copy()
    x[len(x) // 2] = lc.t0 + lc.N          # one past the last row
    bad = workloads.LookupCase(lc.name, x, lc.y, lc.t0, lc.tb, lc.N, lc.lid)
    _say(f"lookup false statement (range) case {k}")
    with pytest.raises(B.VLError) as e:
        B.lookup_prove([lookup_args(bad, "device", to_dev)], seed)
    assert e.value.status == B.VL_ERR_FALSE_STATEMENT


def test_wrong_second_column_is_refused(B):
    cases, seed = _tiny()
    lc, _ = cases[6]
    y = lc.y.copy()
    y[3] += 1
    bad = workloads.LookupCase(lc.name, lc.x, y, lc.t0, lc.tb, lc.N, lc.lid)
    _say("lookup false statement (second column)")
    with pytest.raises(B.VLError) as e:
        B.lookup_prove([lookup_args(bad, "device", to_dev)], seed)
    assert e.value.status == B.VL_ERR_FALSE_STATEMENT
