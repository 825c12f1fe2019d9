"""Host-side checks of the C ABI (no GPU): exports and the CPU verifier.

The library's host verifier (C++ SHA-256 transcript, Montgomery arithmetic,
interpolation and witness MLE evaluation) must accept every proof the oracle
writes and reject every single-element tamper, and its reduced claims must
equal the oracle's challenges and final values.
"""
import json
import os
import re

import numpy as np
import pytest

import oracle
from oracle.zkmat import prove_group, verify_group, Reject
import workloads
from paper_2508_21393_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden")


def _lib_or_skip():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libverilora.so not built")
    return B.lib()


def test_library_exports_every_declared_symbol():
    L = _lib_or_skip()
    header = open(os.path.join(ROOT, "include", "verilora.h")).read()
    declared = set(re.findall(r"\b(vl_[a-z_0-9]+)\s*\(", header))
    assert declared == set(B.EXPORTED)
    for name in declared:
        assert hasattr(L, name), name


def host_group(g: workloads.Group) -> B.GroupArgs:
    prods = [(p.A, p.B, p.transA, p.transB) for p in g.products]
    return B.GroupArgs(g.group_id, prods, g.C)


def _tiny_groups():
    spec = json.load(open(os.path.join(GOLD, "tiny.json")))
    out = []
    for k, (seed, dims, dt, trans, vb) in enumerate(spec["tiny_spec"]):
        g = workloads.tiny_random_group(seed, [tuple(d) for d in dims], dtype=getattr(np, dt),
                                        trans=tuple(trans), value_bits=vb, name=f"tiny{k}")
        g.group_id = k
        out.append((g, bytes.fromhex(spec["groups"][k]["proof_hex"]), spec["seed"]))
    return out


def test_host_verifier_accepts_golden_proofs_with_witness():
    _lib_or_skip()
    cases = _tiny_groups()
    w = workloads.config1()
    cfg1 = json.load(open(os.path.join(GOLD, "cfg1.json")))
    cases.append((w.groups[0], bytes.fromhex(cfg1["groups"][0]["proof_hex"]), w.seed))
    for g, proof, seed in cases:
        ga = host_group(g)
        assert B.proof_size(ga) == len(proof)
        ok, fr, red = B.verify_transcript(proof, ga, seed)
        assert ok, (g.name, B.last_error())
        assert fr == -1
        # reduced claims: c, u, v, then per product r..., a_final, b_final
        res = verify_group(proof, g.shapes, seed, g.group_id)
        expect = [res["c"]] + res["u"] + res["v"]
        for rvec, (af, bf) in zip(res["r"], res["finals"]):
            expect += rvec + [af, bf]
        assert red == expect


def test_host_verifier_rejects_tampering_and_wrong_witness():
    _lib_or_skip()
    g = workloads.tiny_random_group(31, [(6, 10, 5), (6, 3, 5)], trans=(True, False))
    prods = [(p.opA(), p.opB()) for p in g.products]
    proof, _, _ = prove_group(prods, g.C, 77, 0)
    ga = host_group(g)
    assert B.verify_transcript(proof, ga, 77)[0]
    n_el = len(proof) // 32
    for i in range(n_el):
        x = int.from_bytes(proof[32 * i:32 * i + 32], "little")
        bad = proof[:32 * i] + ((x + 1) % oracle.P).to_bytes(32, "little") + proof[32 * i + 32:]
        ok, fr, _ = B.verify_transcript(bad, ga, 77)
        assert not ok, i
        with pytest.raises(Reject):
            verify_group(bad, g.shapes, 77, 0)
    assert not B.verify_transcript(proof, ga, 78)[0]
    assert not B.verify_transcript(proof[:-1], ga, 77)[0]
    assert not B.verify_transcript(proof[:-32] + oracle.P.to_bytes(32, "little"), ga, 77)[0]
    # witness mismatch: same shapes, one entry of C changed
    g2 = workloads.Group(g.name, g.products, g.C.copy(), g.group_id)
    g2.C[0, 0] += 1
    assert not B.verify_transcript(proof, host_group(g2), 77)[0]


def test_round_failure_reports_round_index():
    _lib_or_skip()
    g = workloads.tiny_random_group(5, [(4, 16, 4)])
    prods = [(p.opA(), p.opB()) for p in g.products]
    proof, _, _ = prove_group(prods, g.C, 1, 0)
    ga = B.GroupArgs(0, [(p.A, p.B, p.transA, p.transB) for p in g.products], g.C)
    # change g(0) of round 3 (element 1 + 3*2): rounds 1, 2 pass, round 3 fails
    i = 1 + 3 * 2
    x = int.from_bytes(proof[32 * i:32 * i + 32], "little")
    bad = proof[:32 * i] + ((x + 5) % oracle.P).to_bytes(32, "little") + proof[32 * i + 32:]
    ok, fr, _ = B.verify_transcript(bad, ga, 1)
    assert not ok and fr == 3


# ------------------------------------------------------------ ABI details ---
def test_stage_names_match_the_header():
    header = open(os.path.join(ROOT, "include", "verilora.h")).read()
    defs = dict((k, int(v)) for k, v in re.findall(r"#define (VL_STAGE_[A-Z0-9]+) (\d+)", header))
    assert defs["VL_STAGE_COUNT"] == B.VL_STAGE_COUNT == len(B.STAGE_NAMES)
    assert B.STAGE_NAMES[defs["VL_STAGE_UPLOAD"]] == "upload"
    assert B.STAGE_NAMES[defs["VL_STAGE_EQ"]] == "eq"
    assert B.STAGE_NAMES[defs["VL_STAGE_FINISH"]] == "finish"
    assert B.STAGE_NAMES[defs["VL_STAGE_PASS1"]] == "pass1"
    assert B.STAGE_NAMES[defs["VL_STAGE_ROUNDS"]] == "rounds"
    kinds = defs["VL_STAGE_FINISH"] - defs["VL_STAGE_CONTRACT"]
    assert len(B.STAGE_NAMES[defs["VL_STAGE_CONTRACT"]:defs["VL_STAGE_FINISH"]]) == kinds
    assert f"{kinds} kinds" in header


def test_tuning_struct_matches_the_header():
    header = open(os.path.join(ROOT, "include", "verilora.h")).read()
    end = header.index("} vl_tuning;")
    body = header[header.rindex("typedef struct {", 0, end):end]
    fields = re.findall(r"uint32_t (\w+);", body)
    assert fields == [f for f, _ in B.vl_tuning._fields_]


def _host_args(g: workloads.Group):
    prods = [(p.A, p.B, p.transA, p.transB) for p in g.products]
    return B.GroupArgs(g.group_id, prods, g.C)


def test_prove_refuses_a_misaligned_workspace():
    # refused by the host-side checks, before any device work
    import ctypes
    L = _lib_or_skip()
    ga = _host_args(workloads.tiny_random_group(1, [(4, 4, 4)]))
    opts = B.vl_prove_opts(B.VL_MODE_BATCHED, 0, 0x1000 + 8, 1 << 20, None, None, None)
    proofs = ctypes.create_string_buffer(4096)
    offs = (ctypes.c_uint64 * 2)()
    st = L.vl_sumcheck_matmul_prove(ctypes.byref(ga.struct), 1, 1, ctypes.byref(opts),
                                    ctypes.addressof(proofs), 4096, offs, None, None)
    assert st == B.VL_ERR_WORKSPACE
    assert "256-byte aligned" in B.last_error()


@pytest.mark.parametrize("mode,async_,msg", [(B.VL_MODE_BATCHED, 0, "async must be 1"),
                                             (B.VL_MODE_PER_INSTANCE, 1, "batched mode"),
                                             (B.VL_MODE_PERSISTENT, 1, "batched mode")])
def test_graph_create_refuses_unsupported_options(mode, async_, msg):
    import ctypes
    L = _lib_or_skip()
    ga = _host_args(workloads.tiny_random_group(1, [(4, 4, 4)]))
    opts = B.vl_prove_opts(mode, async_, 0x1000, 1 << 20, 0x2000, None, None)
    offs = (ctypes.c_uint64 * 2)()
    h = ctypes.c_void_p(123)
    st = L.vl_prove_graph_create(ctypes.byref(ga.struct), 1, ctypes.byref(opts), 0x3000, 4096, offs, None,
                                 ctypes.byref(h))
    assert st == B.VL_ERR_INVALID_ARG and msg in B.last_error()
    assert not h.value    # no handle on failure
    L.vl_prove_graph_destroy(None)   # a null handle is a no-op


def test_partial_eval_workspace_refuses_bad_tuning():
    _lib_or_skip()
    assert B.partial_eval_workspace_size(64, 64, 0, np.int16, B.tuning(claim_order=3)) == 0
    assert B.partial_eval_workspace_size(64, 64, 0, np.int16, B.tuning(cols_rows=3)) == 0
    assert B.partial_eval_workspace_size(64, 64, 0, np.int16, B.tuning(claim_order=2)) > 0


def test_persistent_mode_refuses_more_than_128_groups():
    # each resident rounds workgroup fills its CU's register file, so the
    # persistent mode leaves half the CUs to the contractions: the group limit
    # is checked on the host, before any device work
    import ctypes
    L = _lib_or_skip()
    ga = _host_args(workloads.tiny_random_group(1, [(4, 4, 4)]))
    n = 129
    arr = (type(ga.struct) * n)(*([ga.struct] * n))
    opts = B.vl_prove_opts(B.VL_MODE_PERSISTENT, 0, 0x1000, 1 << 20, None, None, None)
    offs = (ctypes.c_uint64 * (n + 1))()
    proofs = ctypes.create_string_buffer(4096)
    st = L.vl_sumcheck_matmul_prove(arr, n, 1, ctypes.byref(opts), ctypes.addressof(proofs), 4096, offs,
                                    None, None)
    assert st == B.VL_ERR_INVALID_ARG
    assert "at most 128 groups" in B.last_error()


BOUNDARY_CALLS = ("vl_fr_lift", "vl_eq_table", "vl_mle_partial_eval", "vl_sumcheck_matmul_prove",
                  "vl_verify_transcript")


def _comment_before(header: str, name: str) -> str:
    """The /* ... */ block that ends right before the declaration of name."""
    decl = re.search(r"\n[a-z_0-9 ]*\b" + name + r"\s*\(", header)
    assert decl, name
    end = header.rindex("*/", 0, decl.start())
    start = header.rindex("/*", 0, end)
    between = header[end + 2:decl.start()]
    assert "/*" not in between and ";" not in between, name
    return header[start:end]


@pytest.mark.parametrize("name", BOUNDARY_CALLS)
def test_boundary_call_cites_the_paper(name):
    # each of the five calls of the boundary says which passage of the paper
    # defines the operation it performs
    header = open(os.path.join(ROOT, "include", "verilora.h")).read()
    comment = _comment_before(header, name)
    assert re.search(r"\bSec\. [IVX]+(-[A-Z](\.\d)?)?|\beq\. \(", comment), name


def test_header_compiles_as_c_and_cpp():
    # the boundary header stands alone for C and C++ callers
    import shutil
    import subprocess
    for cc, lang in (("gcc", "c"), ("g++", "c++")):
        if not shutil.which(cc):
            pytest.skip(f"{cc} not found")
        r = subprocess.run([cc, "-x", lang, "-fsyntax-only", "-Wall", "-Werror",
                            os.path.join(ROOT, "include", "verilora.h")], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="plans with fake device pointers: CPU-only container")
@pytest.mark.parametrize("rows,cols,ld,contract,dt,cols_rows", [
    (130, 777, 784, 1, np.int16, 2), (130, 777, 784, 1, np.int16, 1), (300, 1030, 1032, 1, np.int16, 2),
    (3000, 65, 72, 0, np.int16, 1), (270, 514, 516, 0, np.int32, 1), (300, 301, 302, 0, np.int64, 1),
    (33, 515, 520, 1, np.int32, 1), (9, 4093, 4096, 1, np.int64, 1)])
def test_partial_eval_workspace_size_covers_strided_layouts(rows, cols, ld, contract, dt, cols_rows):
    # the size query knows only (rows, cols): it must cover the plan for any
    # leading dimension and alignment.  The call plans on the host and
    # checks the workspace before any device work; with no GPU here the
    # first launch then fails with VL_ERR_HIP, never with VL_ERR_WORKSPACE.
    import ctypes
    L = _lib_or_skip()
    tn = B.tuning(cols_rows=cols_rows)
    need = B.partial_eval_workspace_size(rows, cols, contract, dt, tn)
    assert need > 0
    len_ = rows if contract == 0 else cols
    n_out = cols if contract == 0 else rows
    eq = B.vl_fr_vec(0x10000, len_, len_)
    out = B.vl_fr_vec(0x20000, n_out, n_out)
    st = L.vl_mle_partial_eval(ctypes.c_void_p(0x100000), B.dtype_code(dt), rows, cols, ld, contract, eq, out,
                               ctypes.c_void_p(0x200000), need, ctypes.byref(tn), None)
    assert st != B.VL_ERR_WORKSPACE, B.last_error()
    assert st == B.VL_ERR_HIP


def _layer_host(w):
    return B.LayerArgs(w)


@pytest.mark.parametrize("dims", [(8, 12, 10, 3), (1, 3, 2, 2), (512, 4096, 11008, 16), (2048, 5120, 13824, 64)])
def test_chain_proof_size_matches_the_oracle(dims):
    from oracle.chain import chain_proof_len
    _lib_or_skip()
    T, d_in, d_out, r = dims
    st = B.vl_lora_layer(T, d_in, d_out, r, 12, 3, *([0] * 15))
    assert B.lib().vl_lora_chain_proof_size(ctypes_byref(st)) == chain_proof_len(dims)
    assert B.lib().vl_lora_chain_workspace_size(ctypes_byref(st)) > 0


def ctypes_byref(x):
    import ctypes
    return ctypes.byref(x)


def test_chain_refuses_bad_layers_before_device_work():
    import ctypes
    L = _lib_or_skip()
    st = B.vl_lora_layer(8, 12, 10, 3, 12, 3, *([0x1000] * 15))
    buf = ctypes.create_string_buffer(64)
    # proof buffer too small: refused on the host
    assert L.vl_lora_chain_prove(ctypes.byref(st), 1, 0x10000, 1 << 20, ctypes.addressof(buf), 64, None,
                                 None) == B.VL_ERR_BUFFER_TOO_SMALL
    st2 = B.vl_lora_layer(8, 12, 10, 3, 12, 3, *([0x1000] * 14 + [0]))
    assert L.vl_lora_chain_prove(ctypes.byref(st2), 1, 0x10000, 1 << 20, ctypes.addressof(buf), 64, None,
                                 None) == B.VL_ERR_INVALID_ARG
    st3 = B.vl_lora_layer(70000, 12, 10, 3, 12, 3, *([0x1000] * 15))
    assert L.vl_lora_chain_proof_size(ctypes.byref(st3)) == 0
