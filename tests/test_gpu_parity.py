"""Parity of the HIP prover with the CPU oracle (needs a gfx950 GPU).

Every comparison is exact: field elements and proof bytes must be identical
to what the oracle computes on the same seeded inputs (tolerance 0).  Small
cases compare against the oracle directly; full-size configs compare proof
digests stored by tests/golden/make_golden.py (oracle runs).
"""
import random
import sys

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import device_group, golden, sha, tiny_workload, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_21393_amd import binding
    binding.lib()  # raises if the library is missing: no fallback
    return binding


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _export(B, vec_t, n):
    import torch
    out = torch.empty((n, 8), dtype=torch.int32, device="cuda")
    B.fr_export(B.fr_vec(vec_t, n), n, out)
    torch.cuda.synchronize()
    w = out.cpu().numpy().astype(np.uint32).astype(object)
    return [sum(int(w[i, j]) << (32 * j) for j in range(8)) for i in range(n)]


@pytest.mark.parametrize("dtype,bits", [(np.int16, 15), (np.int32, 31), (np.int64, 62)])
def test_fr_lift(B, dtype, bits):
    import torch
    rng = np.random.default_rng(1)
    n = 1000
    x = rng.integers(-(1 << bits), 1 << bits, size=n, dtype=np.int64).astype(dtype)
    x[:3] = [0, -1, 1]
    vec = torch.empty((8, n), dtype=torch.int32, device="cuda")
    B.fr_lift(to_dev(x), n, B.fr_vec(vec))
    assert _export(B, vec, n) == [oracle.lift(int(v)) for v in x]


@pytest.mark.parametrize("n", [0, 1, 5, 11])
def test_eq_table(B, n):
    import torch
    rng = random.Random(n)
    pt = [rng.randrange(oracle.P) for _ in range(n)]
    L = 1 << n
    vec = torch.empty((8, L), dtype=torch.int32, device="cuda")
    B.eq_table(pt, B.fr_vec(vec))
    assert _export(B, vec, L) == oracle.eq_table(pt)


PE_CASES = [
    # rows, cols, contract, dtype, bits
    (1, 1, 0, np.int16, 15), (7, 3, 0, np.int16, 15), (300, 130, 0, np.int16, 15),
    (5, 1000, 1, np.int16, 15), (130, 777, 1, np.int16, 15), (64, 2048, 1, np.int16, 15),
    (3000, 65, 0, np.int16, 15), (33, 515, 1, np.int32, 31), (40, 77, 0, np.int64, 62),
    (17, 260, 1, np.int64, 40), (9, 4096, 1, np.int64, 44),
    # vector rows kernels of wide entries: 4 int32 or 2 int64 columns per lane
    # (16-byte loads), ragged column groups and row tails
    (270, 516, 0, np.int32, 31), (300, 302, 0, np.int64, 62), (37, 1024, 0, np.int64, 62),
]


@pytest.mark.parametrize("rows,cols,contract,dtype,bits", PE_CASES)
def test_mle_partial_eval(B, rows, cols, contract, dtype, bits):
    import torch
    _say(f"partial_eval rows={rows} cols={cols} contract={contract} dtype={dtype.__name__}")
    rng = np.random.default_rng(rows * 7919 + cols)
    M = rng.integers(-(1 << bits), 1 << bits, size=(rows, cols), dtype=np.int64).astype(dtype)
    len_ = rows if contract == 0 else cols
    nv = oracle.num_vars(len_)
    prng = random.Random(len_)
    pt = [prng.randrange(oracle.P) for _ in range(nv)]
    eq = torch.empty((8, 1 << nv), dtype=torch.int32, device="cuda")
    B.eq_table(pt, B.fr_vec(eq))
    n_out = cols if contract == 0 else rows
    L = 1 << oracle.num_vars(n_out)
    out = torch.full((8, L), 7, dtype=torch.int32, device="cuda")
    ws = torch.empty(B.partial_eval_workspace_size(rows, cols, contract, M.dtype), dtype=torch.uint8,
                     device="cuda")
    B.mle_partial_eval(to_dev(M), contract, B.fr_vec(eq), B.fr_vec(out), ws)
    got = _export(B, out, L)
    if contract == 0:
        expect = oracle.partial_eval_rows(M, pt)
    else:
        expect = oracle.partial_eval_cols(M, pt)
    assert got == expect


@pytest.mark.parametrize("rows,cols,ld,lane_macs", [(67, 1003, 1024, 2048), (130, 517, 520, 0), (9, 77, 80, 512)])
def test_mle_partial_eval_strided_cols(B, rows, cols, ld, lane_macs):
    # a strided view (ld > cols, rows 16-byte aligned) contracted over its
    # columns: ragged stages and a last piece of fewer than 8 entries, in
    # chunks of a few hundred entries
    import torch
    _say(f"partial_eval strided rows={rows} cols={cols} ld={ld} lane_macs={lane_macs}")
    rng = np.random.default_rng(rows * 31 + cols)
    big = rng.integers(-(1 << 15), 1 << 15, size=(rows, ld), dtype=np.int64).astype(np.int16)
    Md = to_dev(big)[:, :cols]
    nv = oracle.num_vars(cols)
    prng = random.Random(cols)
    pt = [prng.randrange(oracle.P) for _ in range(nv)]
    eq = torch.empty((8, 1 << nv), dtype=torch.int32, device="cuda")
    B.eq_table(pt, B.fr_vec(eq))
    L = 1 << oracle.num_vars(rows)
    out = torch.full((8, L), 7, dtype=torch.int32, device="cuda")
    tn = B.tuning(lane_macs=lane_macs) if lane_macs else None
    ws = torch.empty(B.partial_eval_workspace_size(rows, cols, 1, np.int16, tn), dtype=torch.uint8, device="cuda")
    B.mle_partial_eval(Md, 1, B.fr_vec(eq), B.fr_vec(out), ws, tuning_=tn)
    assert _export(B, out, L) == oracle.partial_eval_cols(big[:, :cols], pt)


@pytest.mark.parametrize("rows,cols,ld", [(130, 777, 784), (256, 4096, 4096), (300, 1030, 1032), (129, 64, 64)])
def test_mle_partial_eval_cols_two_rows_per_lane(B, rows, cols, ld):
    # vl_tuning.cols_rows = 2: the int16 column kernel with two rows per lane
    # (reached only through tuning), ragged last row pair and strided rows
    import torch
    _say(f"partial_eval cols_rows=2 rows={rows} cols={cols} ld={ld}")
    rng = np.random.default_rng(rows * 13 + cols)
    big = rng.integers(-(1 << 15), 1 << 15, size=(rows, ld), dtype=np.int64).astype(np.int16)
    Md = to_dev(big)[:, :cols]
    nv = oracle.num_vars(cols)
    prng = random.Random(cols + 1)
    pt = [prng.randrange(oracle.P) for _ in range(nv)]
    eq = torch.empty((8, 1 << nv), dtype=torch.int32, device="cuda")
    B.eq_table(pt, B.fr_vec(eq))
    L = 1 << oracle.num_vars(rows)
    out = torch.full((8, L), 7, dtype=torch.int32, device="cuda")
    tn = B.tuning(cols_rows=2)
    ws = torch.empty(B.partial_eval_workspace_size(rows, cols, 1, np.int16, tn), dtype=torch.uint8, device="cuda")
    B.mle_partial_eval(Md, 1, B.fr_vec(eq), B.fr_vec(out), ws, tuning_=tn)
    assert _export(B, out, L) == oracle.partial_eval_cols(big[:, :cols], pt)


def _prove(B, w, mode):
    gs = [device_group(g, B) for g in w.groups]
    return B.sumcheck_matmul_prove(gs, w.seed, mode=mode)


@pytest.mark.parametrize("mode", [0, 1])
def test_tiny_cases_match_oracle_bytes(B, mode):
    w, spec = tiny_workload()
    _say(f"tiny cases mode={mode}")
    proofs, digests = _prove(B, w, mode)
    for g, pr, dg, gold in zip(w.groups, proofs, digests, spec["groups"]):
        assert pr.hex() == gold["proof_hex"], g.name
        assert dg.hex() == gold["state"], g.name


@pytest.mark.parametrize("mode", [0, 1])
def test_cfg1_matches_oracle(B, mode):
    w = workloads.config1()
    gold = golden("cfg1")["groups"][0]
    proofs, digests = _prove(B, w, mode)
    assert proofs[0].hex() == gold["proof_hex"]
    assert digests[0].hex() == gold["state"]
    ga = device_group(w.groups[0], B)
    host = B.GroupArgs(0, [(p.A, p.B, p.transA, p.transB) for p in w.groups[0].products], w.groups[0].C)
    ok, fr, _ = B.verify_transcript(proofs[0], host, w.seed)
    assert ok and fr == -1
    del ga


def test_cfg1_seed_sweep_batched(B):
    sweep = golden("cfg1_sweep")
    gs, expect = [], []
    for i, rec in enumerate(sweep):
        w = workloads.config1(seed=rec["seed"])
        g = w.groups[0]
        gs.append((g, rec["seed"], rec["groups"][0]["proof_hex"]))
    # every seed is its own call (a seed keys the transcript of all groups in a call)
    for g, seed, hx in gs:
        proofs, _ = B.sumcheck_matmul_prove([device_group(g, B)], seed, mode=1)
        assert proofs[0].hex() == hx


def test_batch_is_order_independent(B):
    w, spec = tiny_workload()
    gs = [device_group(g, B) for g in w.groups]
    order = list(range(len(gs)))[::-1]
    proofs, _ = B.sumcheck_matmul_prove([gs[i] for i in order], w.seed, mode=1)
    for i, pr in zip(order, proofs):
        assert pr.hex() == spec["groups"][i]["proof_hex"]


def test_false_statement_refused(B):
    g = workloads.tiny_random_group(3, [(8, 8, 8)])
    g.C = g.C.copy()
    g.C[7, 0] += 1
    with pytest.raises(B.VLError) as e:
        B.sumcheck_matmul_prove([device_group(g, B)], 1, mode=1)
    assert e.value.status == B.VL_ERR_FALSE_STATEMENT


def test_range_error_on_oversized_claim_entry(B):
    # an int64 C entry beyond three 16-bit digits is refused, not mis-proved
    g = workloads.tiny_random_group(4, [(4, 4, 4)])
    g.C = g.C.copy()
    g.C[1, 1] = 1 << 60
    with pytest.raises(B.VLError) as e:
        B.sumcheck_matmul_prove([device_group(g, B)], 1, mode=1)
    assert e.value.status == B.VL_ERR_RANGE


def test_range_error_in_row_order_claim(B):
    # C with 256 columns is contracted over its rows (two columns per lane,
    # 16-byte loads): an entry outside |x| < 2^47 there is refused as well
    g = workloads.tiny_random_group(5, [(8, 8, 256)])
    g.C = g.C.copy()
    g.C[3, 201] = 1 << 60
    with pytest.raises(B.VLError) as e:
        B.sumcheck_matmul_prove([device_group(g, B)], 1, mode=1)
    assert e.value.status == B.VL_ERR_RANGE


@pytest.mark.parametrize("order", [1, 2])
def test_claim_order_matches_oracle_bytes(B, order):
    # the claim contracted over the columns of C (order 1) or over its rows
    # (order 2) for every tiny case: same proof bytes
    w, spec = tiny_workload()
    _say(f"tiny cases claim_order={order}")
    gs = [device_group(g, B) for g in w.groups]
    proofs, digests = B.sumcheck_matmul_prove(gs, w.seed, mode=1, tuning_=B.tuning(claim_order=order))
    for g, pr, dg, gold in zip(w.groups, proofs, digests, spec["groups"]):
        assert pr.hex() == gold["proof_hex"], g.name
        assert dg.hex() == gold["state"], g.name


def test_two_rows_per_lane_tiny_cases(B):
    # cols_rows = 2 with the claim over the columns of C: the int16 and the
    # two-digit int64 column kernels with two rows per lane where a
    # contraction has >= 128 outputs
    w, spec = tiny_workload()
    _say("tiny cases cols_rows=2 claim_order=1")
    gs = [device_group(g, B) for g in w.groups]
    proofs, digests = B.sumcheck_matmul_prove(gs, w.seed, mode=1, tuning_=B.tuning(cols_rows=2, claim_order=1))
    for g, pr, dg, gold in zip(w.groups, proofs, digests, spec["groups"]):
        assert pr.hex() == gold["proof_hex"], g.name
        assert dg.hex() == gold["state"], g.name


@pytest.mark.parametrize("knobs", [dict(cols_rows=2, claim_order=1), dict(lane_macs=4096),
                                   dict(lane_macs=16384), dict(contract_streams=1),
                                   dict(contract_streams=2, segments=3)])
def test_tuned_launch_shapes_full_size_cfg3(B, knobs):
    # launch shapes the autotuner may pick, at full size: the proof bytes
    # must still be the oracle's
    _say(f"cfg3 tuned {knobs}: generating")
    w = workloads.make_config("cfg3")
    gold = golden("cfg3")
    gs = [device_group(g, B) for g in w.groups]
    _say(f"cfg3 tuned {knobs}: proving")
    proofs, digests = B.sumcheck_matmul_prove(gs, w.seed, mode=1, tuning_=B.tuning(**knobs))
    for g, pr, dg, rec in zip(w.groups, proofs, digests, gold["groups"]):
        assert sha(pr) == rec["proof_sha256"], g.name
        assert dg.hex() == rec["state"], g.name


def test_claim_order_full_size_cfg3(B):
    _say("cfg3 claim orders: generating")
    w = workloads.make_config("cfg3")
    gold = golden("cfg3")
    gs = [device_group(g, B) for g in w.groups]
    for order in (1, 2):
        _say(f"cfg3: proving, claim_order={order}")
        proofs, digests = B.sumcheck_matmul_prove(gs, w.seed, mode=1, tuning_=B.tuning(claim_order=order))
        for g, pr, dg, rec in zip(w.groups, proofs, digests, gold["groups"]):
            assert sha(pr) == rec["proof_sha256"], g.name
            assert dg.hex() == rec["state"], g.name


def test_async_prove_into_device_buffers(B):
    import torch
    w, spec = tiny_workload()
    gs = [device_group(g, B) for g in w.groups]
    total = sum(B.proof_size(g) for g in gs)
    proofs = torch.zeros(total, dtype=torch.uint8, device="cuda")
    status = torch.full((len(gs),), -1, dtype=torch.int32, device="cuda")
    ws = torch.empty(B.workspace_size(gs, 1, async_=True), dtype=torch.uint8, device="cuda")
    offs = B.sumcheck_matmul_prove_async(gs, w.seed, proofs, status, ws, mode=1)
    torch.cuda.synchronize()
    raw = proofs.cpu().numpy().tobytes()
    assert status.cpu().tolist() == [0] * len(gs)
    for i, gold in enumerate(spec["groups"]):
        assert raw[offs[i]:offs[i + 1]].hex() == gold["proof_hex"]


def test_async_prove_into_pinned_host_buffers(B):
    # the kernels write proofs, status words and digests straight into pinned
    # host memory; a slice at an offset checks interior pointers too
    import torch
    w, spec = tiny_workload()
    gs = [device_group(g, B) for g in w.groups]
    total = sum(B.proof_size(g) for g in gs)
    buf = torch.zeros(total + 256, dtype=torch.uint8, pin_memory=True)
    proofs = buf[256:]
    status = torch.full((len(gs),), -1, dtype=torch.int32, pin_memory=True)
    digests = torch.zeros(32 * len(gs), dtype=torch.uint8, pin_memory=True)
    ws = torch.empty(B.workspace_size(gs, 1, async_=True), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    offs = B.sumcheck_matmul_prove_async(gs, w.seed, proofs, status, ws, mode=1, digests_dev=digests, stream=s)
    s.synchronize()
    assert status.tolist() == [0] * len(gs)
    raw = proofs.numpy().tobytes()
    dg = digests.numpy().tobytes()
    assert not buf[:256].any()
    for i, gold in enumerate(spec["groups"]):
        assert raw[offs[i]:offs[i + 1]].hex() == gold["proof_hex"]
        assert dg[32 * i:32 * i + 32].hex() == gold["state"]


def test_async_refuses_pageable_host_buffers(B):
    import torch
    w, _ = tiny_workload()
    gs = [device_group(g, B) for g in w.groups[:1]]
    proofs = torch.zeros(B.proof_size(gs[0]), dtype=torch.uint8)        # pageable
    status = torch.zeros(1, dtype=torch.int32, pin_memory=True)
    ws = torch.empty(B.workspace_size(gs, 1, async_=True), dtype=torch.uint8, device="cuda")
    with pytest.raises(B.VLError) as e:
        B.sumcheck_matmul_prove_async(gs, w.seed, proofs, status, ws, mode=1)
    assert e.value.status == B.VL_ERR_INVALID_ARG


@pytest.mark.parametrize("cfg", ["cfg2", "cfg3", "cfg4"])
def test_full_size_config_matches_oracle(B, cfg):
    # blocking calls: the large contraction kinds run on two streams
    _say(f"{cfg}: generating")
    # the 7B block's witness products run as float64 GEMMs on the GPU (exact:
    # all partial sums are integers below 2^53); the others on the host
    w = workloads.make_config(cfg, **({"device": "cuda"} if cfg == "cfg4" else {}))
    gold = golden(cfg)
    _say(f"{cfg}: proving {len(w.groups)} groups")
    proofs, digests = _prove(B, w, 1)
    for g, pr, dg, rec in zip(w.groups, proofs, digests, gold["groups"]):
        assert rec["name"] == g.name
        assert sha(pr) == rec["proof_sha256"], g.name
        assert dg.hex() == rec["state"], g.name


def test_async_full_size_cfg4_long_row_chunks(B):
    # an asynchronous call on a batch that streams over 1 GB (the 7B block,
    # 3.8 GB) contracts its int16 matrices over rows in chunks 16 times
    # longer than a blocking call does (fewer chunk sums for the finish
    # pass); its proofs must still be the oracle's bytes
    import torch
    _say("cfg4 async: generating")
    w = workloads.make_config("cfg4", device="cuda")
    gold = golden("cfg4")
    gs = [device_group(g, B) for g in w.groups]
    total = sum(B.proof_size(g) for g in gs)
    async_ws = B.workspace_size(gs, 1, async_=True)
    # an explicit lane_macs keeps the short chunks: more room for chunk sums
    assert async_ws < B.workspace_size(gs, 1, async_=True, tuning_=B.tuning(lane_macs=8192))
    proofs = torch.zeros(total, dtype=torch.uint8, device="cuda")
    status = torch.full((len(gs),), -1, dtype=torch.int32, device="cuda")
    ws = torch.empty(async_ws, dtype=torch.uint8, device="cuda")
    _say(f"cfg4 async: proving {len(gs)} groups")
    offs = B.sumcheck_matmul_prove_async(gs, w.seed, proofs, status, ws, mode=1)
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [0] * len(gs)
    raw = proofs.cpu().numpy().tobytes()
    for i, (g, rec) in enumerate(zip(w.groups, gold["groups"])):
        assert sha(raw[offs[i]:offs[i + 1]]) == rec["proof_sha256"], g.name


# ------------------------------------------------------------ graph mode ---
@pytest.mark.parametrize("segments", [1, 3])
def test_prove_graph_replays_match_eager(B, segments):
    # one capture, replayed for several seeds with eager proves (their own
    # launches and synchronisations) in between; every replay must equal the
    # eager proof of its seed, and the workload's seed its oracle bytes
    import torch
    w, spec = tiny_workload()
    gs = [device_group(g, B) for g in w.groups]
    total = sum(B.proof_size(g) for g in gs)
    proofs = torch.zeros(total, dtype=torch.uint8, device="cuda")
    status = torch.full((len(gs),), -1, dtype=torch.int32, device="cuda")
    digests = torch.zeros(32 * len(gs), dtype=torch.uint8, device="cuda")
    tn = B.tuning(segments=segments)
    ws = torch.empty(B.workspace_size(gs, 1, async_=True, tuning_=tn), dtype=torch.uint8, device="cuda")
    _say(f"prove graph segments={segments}")
    with B.ProveGraph(gs, ws, proofs, status, digests_dev=digests, tuning_=tn) as G:
        for seed in (w.seed, 7, 7, w.seed + 1, w.seed):
            proofs.zero_()
            status.fill_(-1)
            G.launch(seed)
            torch.cuda.synchronize()
            assert status.cpu().tolist() == [0] * len(gs)
            raw = proofs.cpu().numpy().tobytes()
            dg = digests.cpu().numpy().tobytes()
            ref, ref_dig = B.sumcheck_matmul_prove(gs, seed, mode=1)
            for i in range(len(gs)):
                assert raw[G.offsets[i]:G.offsets[i + 1]] == ref[i], (seed, i)
                assert dg[32 * i:32 * i + 32] == ref_dig[i], (seed, i)
            if seed == w.seed:
                for i, gold in enumerate(spec["groups"]):
                    assert raw[G.offsets[i]:G.offsets[i + 1]].hex() == gold["proof_hex"]


@pytest.mark.parametrize("streams", [0, 2])
def test_prove_graph_full_size_cfg3(B, streams):
    # streams 2: the contraction kinds (each above 100 MB here) forked over
    # two streams inside the captured graph; 0: the default (one stream)
    import torch
    _say(f"cfg3 graph streams={streams}: generating")
    w = workloads.make_config("cfg3")
    gold = golden("cfg3")
    gs = [device_group(g, B) for g in w.groups]
    total = sum(B.proof_size(g) for g in gs)
    proofs = torch.empty(total, dtype=torch.uint8, pin_memory=True)
    status = torch.empty(len(gs), dtype=torch.int32, pin_memory=True)
    tn = B.tuning(contract_streams=streams)
    ws = torch.empty(B.workspace_size(gs, 1, async_=True, tuning_=tn), dtype=torch.uint8, device="cuda")
    with B.ProveGraph(gs, ws, proofs, status, tuning_=tn) as G:
        for rep in range(3):
            _say(f"cfg3 graph streams={streams}: replay {rep}")
            proofs.numpy()[:] = 0
            G.launch(w.seed)
            torch.cuda.synchronize()
            assert not status.numpy().any()
            raw = proofs.numpy().tobytes()
            for i, (g, rec) in enumerate(zip(w.groups, gold["groups"])):
                assert sha(raw[G.offsets[i]:G.offsets[i + 1]]) == rec["proof_sha256"], g.name
            x = torch.randn(1 << 20, device="cuda")   # eager work between the replays
            (x * 2).sum().item()


def test_prove_graph_owns_its_descriptors(B):
    # the caller's product descriptors are overwritten (every field zero)
    # after create: the graph keeps its own copies, so its launches still
    # prove the same matrices
    import torch
    w, spec = tiny_workload()
    gs = [device_group(g, B) for g in w.groups]
    batch = B.GroupBatch(gs)
    total = batch.total
    proofs = torch.zeros(total, dtype=torch.uint8, device="cuda")
    status = torch.full((len(gs),), -1, dtype=torch.int32, device="cuda")
    ws = torch.empty(B.workspace_size(batch, 1, async_=True), dtype=torch.uint8, device="cuda")
    _say("prove graph: descriptors overwritten after create")
    with B.ProveGraph(batch, ws, proofs, status) as G:
        for ga in gs:
            for k in range(len(ga.prods)):
                ga.prods[k] = B.vl_product()
        for i in range(len(batch.arr)):
            batch.arr[i] = B.vl_group()
        for rep in range(2):
            proofs.zero_()
            G.launch(w.seed)
            torch.cuda.synchronize()
            assert status.cpu().tolist() == [0] * len(gs)
            raw = proofs.cpu().numpy().tobytes()
            for i, gold in enumerate(spec["groups"]):
                assert raw[G.offsets[i]:G.offsets[i + 1]].hex() == gold["proof_hex"], (rep, i)


@pytest.mark.parametrize("mode", [0, 2])
def test_prove_graph_refuses_other_modes(B, mode):
    import torch
    w, _ = tiny_workload()
    gs = [device_group(g, B) for g in w.groups[:1]]
    proofs = torch.zeros(B.proof_size(gs[0]), dtype=torch.uint8, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = torch.empty(B.workspace_size(gs, mode, async_=True), dtype=torch.uint8, device="cuda")
    with pytest.raises(B.VLError) as e:
        B.ProveGraph(gs, ws, proofs, status, mode=mode)
    assert e.value.status == B.VL_ERR_INVALID_ARG


# --------------------------------------------------------------- persistent --
def test_persistent_mode_matches_oracle_bytes(B):
    # resident rounds workgroups waiting on readiness counters: same bytes
    w, spec = tiny_workload()
    _say("tiny cases mode=persistent")
    proofs, digests = _prove(B, w, B.VL_MODE_PERSISTENT)
    for g, pr, dg, gold in zip(w.groups, proofs, digests, spec["groups"]):
        assert pr.hex() == gold["proof_hex"], g.name
        assert dg.hex() == gold["state"], g.name


def test_persistent_mode_full_size_cfg3(B):
    _say("cfg3 persistent: generating")
    w = workloads.make_config("cfg3")
    gold = golden("cfg3")
    for segments in (1, 4):
        _say(f"cfg3 persistent: proving, {segments} segments")
        gs = [device_group(g, B) for g in w.groups]
        proofs, digests = B.sumcheck_matmul_prove(gs, w.seed, mode=B.VL_MODE_PERSISTENT,
                                                  tuning_=B.tuning(segments=segments))
        for g, pr, dg, rec in zip(w.groups, proofs, digests, gold["groups"]):
            assert sha(pr) == rec["proof_sha256"], g.name
            assert dg.hex() == rec["state"], g.name


def test_persistent_calls_in_flight_fall_back_to_batched(B):
    # two asynchronous persistent calls on two streams: the second finds the
    # first still running on the device (or not; either way) and both prove
    # the oracle's bytes
    import torch
    w, spec = tiny_workload()
    gs = [device_group(g, B) for g in w.groups]
    batch = B.GroupBatch(gs)
    outs = []
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    _say("persistent: two calls in flight")
    for s in streams:
        proofs = torch.zeros(batch.total, dtype=torch.uint8, device="cuda")
        status = torch.full((len(gs),), -1, dtype=torch.int32, device="cuda")
        ws = torch.empty(B.workspace_size(batch, B.VL_MODE_PERSISTENT, async_=True), dtype=torch.uint8,
                         device="cuda")
        offs = B.sumcheck_matmul_prove_async(batch, w.seed, proofs, status, ws, mode=B.VL_MODE_PERSISTENT,
                                             stream=s)
        outs.append((proofs, status, offs, ws))
    torch.cuda.synchronize()
    for proofs, status, offs, _ in outs:
        assert status.cpu().tolist() == [0] * len(gs)
        raw = proofs.cpu().numpy().tobytes()
        for i, gold in enumerate(spec["groups"]):
            assert raw[offs[i]:offs[i + 1]].hex() == gold["proof_hex"]


def test_persistent_spin_limit_reports_timeout(B):
    # a spin limit of one poll (forced from the host): the resident rounds
    # give up long before the contractions are done, report VL_ERR_TIMEOUT,
    # and every kernel still exits normally
    g = workloads.tiny_random_group(11, [(512, 4096, 512)])
    _say("persistent timeout")
    with pytest.raises(B.VLError) as e:
        B.sumcheck_matmul_prove([device_group(g, B)], 1, mode=B.VL_MODE_PERSISTENT,
                                tuning_=B.tuning(spin_limit=1))
    assert e.value.status == B.VL_ERR_TIMEOUT
    # the same call with the default limit proves
    proofs, _ = B.sumcheck_matmul_prove([device_group(g, B)], 1, mode=B.VL_MODE_PERSISTENT)
    ref, _ = B.sumcheck_matmul_prove([device_group(g, B)], 1, mode=B.VL_MODE_BATCHED)
    assert proofs == ref
