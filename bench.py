#!/usr/bin/env python3
"""Benchmark of the matmul-sumcheck prover on one MI355X.

Workload: one 7B-class decoder block (hidden 4096, FFN 11008, 32 heads) at
T = 2048 tokens with rank-16 LoRA on q, k, v, o, gate, up and down: every
forward, backward and LoRA-update product, 56 products in 49 groups, int16
operands and exact int64 outputs (seeded synthetic data, ``workloads``).  A
step proves all 49 groups in one call with inputs resident in HBM and the
proof bytes copied back to the host.  Throughput (value, ms_per_step) is
measured with --inflight proofs in flight on separate streams (the
asynchronous entry point); latency and per-stage device times with one
blocking call at a time.

Reports (one JSON line): algorithmic Fr MACs/s (value), proofs/s, p50/p99
step latency, the per-instance prover on the same inputs, the dominant
kernel against the HBM roofline (algorithmic matrix bytes over its
HIP-event launch time in the timed steps) with every contraction kind's
GB/s and fraction of the 32-bit multiply peak, and the CPU oracle on the
same block (every group, one worker process per host core).
"""
import argparse
import gc
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# Hardware queues for this process, read when the runtime starts (before any
# GPU call): HIP gives a stream a queue at its first launch, and with its
# default of 4 the proofs in flight, the caller's stream and the library's
# side stream share queues, so one proof's sumcheck rounds can hold up
# another's contractions.  16 gives every stream its own queue (a larger
# value set by the caller is kept).
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4) < 16:
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

METRIC = "Fr MACs/s + matmul-sumcheck proofs/s; batched vs per-instance; p50/p99 latency"
CU, LANES_PER_CLK, CLOCK_HZ = 256, 64, 2.4e9   # MI355X: CUs, VALU lanes per CU per clock, peak clock
HBM_GBPS = 8000.0                               # MI355X HBM3E peak
# v_mad_i64_i32 per matrix entry: 8 eq digits x the entry's digits
MAD_PER_ENTRY = {"i16_rows": 8, "i16_rows4_vec": 8, "i16_cols_vec": 8, "i16_cols2_vec": 8,
                 "i64s_cols_vec": 16, "i64s_cols2_vec": 16, "i64s_rows2_vec": 16, "i64s_rows": 16}


def nv(d):
    return max(0, math.ceil(math.log2(d))) if d > 1 else 0


def algorithmic_macs(shapes_by_group):
    """Fr multiply-accumulates the method needs (partial evaluations, claim,
    rounds and folds, eq tables), independent of how the kernels do them."""
    total = 0
    for shapes in shapes_by_group:
        d0, _, d2 = shapes[0]
        total += d0 * d2 + d0 + (2 ** nv(d0) - 1) + (2 ** nv(d2) - 1)
        for (a, b, c) in shapes:
            total += a * b + b * c + 5 * (2 ** nv(b) - 1)
    return total


def contraction_bytes(groups, cols_rows=1, claim_order=0):
    """Matrix bytes and entries streamed per prove call by each contraction
    kernel kind (stage index -> (bytes, entries)), following the library's
    planning rule for these operands (int16 A and B, int64 C with
    |C| < 2^47, all 16-byte aligned): a row contraction with at least 256
    outputs runs 4 columns per lane with 8-byte loads, else 1 column per
    lane; column contractions read 16-byte vectors, two rows per lane when
    tuned so and there are >= 128 rows; C is contracted over its rows (two
    columns per lane, 16-byte loads) when it has >= 256 columns or when
    tuned so, else over its columns."""
    from paper_2508_21393_amd import binding as B
    k = {}

    def add(name, entries, esize):
        b, e = k.get(name, (0, 0))
        k[name] = (b + entries * esize, e + entries)

    def cols16(n_out):
        return "i16_cols2_vec" if cols_rows == 2 and n_out >= 128 else "i16_cols_vec"

    for g in groups:
        d0, _, d2 = g.products[0].dims
        if claim_order == 2 or (claim_order == 0 and d2 >= 256):
            add("i64s_rows2_vec" if d2 >= 128 else "i64s_rows", d0 * d2, 8)
        else:
            add("i64s_cols2_vec" if cols_rows == 2 and d0 >= 128 else "i64s_cols_vec", d0 * d2, 8)
        for p in g.products:
            d0, d1, d2 = p.dims
            # A side: outputs are the D1 columns of op(A)
            if p.transA:
                add(cols16(d1), d0 * d1, 2)
            else:
                add("i16_rows4_vec" if d1 >= 256 else "i16_rows", d0 * d1, 2)
            # B side: outputs are the D1 rows of op(B)
            if p.transB:
                add("i16_rows4_vec" if d1 >= 256 else "i16_rows", d1 * d2, 2)
            else:
                add(cols16(d1), d1 * d2, 2)
    return {B.STAGE_NAMES.index(n): v for n, v in k.items() if v[1]}


CONTRACT_SOURCES = ("contract.hip", "device.hpp", "contract_job.hpp", "fr.hpp")


def contract_source_sha256():
    """Fingerprint of the contraction kernels' source: the files they are
    compiled from, in a fixed order."""
    import hashlib
    h = hashlib.sha256()
    for name in CONTRACT_SOURCES:
        with open(os.path.join(ROOT, "paper_2508_21393_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(stage_name):
    """HBM bytes per launch of a contraction kind from the rocprofv3 counter
    summary in profiles/, or None when there is none for this kind or the
    contraction source changed since the counters were taken."""
    import glob
    import re
    h = contract_source_sha256()
    for path in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.md")):
        m = re.search(r"```json\s*(\{.*?\})\s*```", open(path).read(), re.S)
        if not m:
            continue
        rec = json.loads(m.group(1))
        if rec.get("stage") == stage_name and rec.get("contract_source_sha256") == h:
            return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    return None


_CPU_W = None


def _cpu_prove(i):
    from oracle.zkmat import prove_workload_group
    g = _CPU_W.groups[i]
    t = time.perf_counter()
    prove_workload_group(g, _CPU_W.seed)
    return i, time.perf_counter() - t


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores(cap=16):
    """CPU threads this process may use: its affinity set, at most `cap`
    (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def cpu_baseline(workload, procs=None):
    """The oracle, unmodified, on every group of the same block: one process
    per host core (forked workers that share the witness arrays), largest
    groups first, wall time from the first group to the last.  Witness
    generation is not timed.  The workers only run Python integer arithmetic
    and hashlib (nothing touches the GPU)."""
    import multiprocessing as mp
    import oracle  # noqa: F401
    global _CPU_W
    _CPU_W = workload
    procs = procs or host_cores()
    order = sorted(range(len(workload.groups)), key=lambda i: -algorithmic_macs([workload.groups[i].shapes]))
    macs = algorithmic_macs([g.shapes for g in workload.groups])
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs) as pool:
        res = pool.map(_cpu_prove, order, chunksize=1)
    dt = time.perf_counter() - t0
    busy = sum(t for _, t in res)
    return {"value": macs / dt, "unit": "Fr-MAC/s", "cores": procs, "kind": "oracle",
            "sample": f"{len(res)} of {len(workload.groups)} groups of the same block (the whole block, "
                      f"{macs / 1e6:.1f} M MACs) in {dt:.1f} s wall on {procs} worker processes "
                      f"({busy:.1f} core-s of proving, {macs / busy / 1e6:.1f} M Fr-MAC/s per core); "
                      f"host CPU: {cpu_model()}, {os.cpu_count()} logical CPUs visible, "
                      f"{host_cores(1 << 30)} in this process's affinity set"}


def peak_rates():
    import ctypes
    from paper_2508_21393_amd.build import PEAK_LIB
    if not os.path.exists(PEAK_LIB):
        return None
    L = ctypes.CDLL(PEAK_LIB)
    L.vlpeak_lane_ops_per_s.restype = ctypes.c_double
    L.vlpeak_lane_ops_per_s.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32]
    names = ["dot2_i32_i16", "mad_u64_u32", "mul_lo_u32", "mul_hi_u32", "add_u32", "mad_i64_i32"]
    return {n: L.vlpeak_lane_ops_per_s(i, 8192, 4096) for i, n in enumerate(names)}


def streaming_read_GBps(nbytes=4 << 30):
    """A plain 16-byte streaming read of a 4 GiB device buffer (libvlpeak.so):
    the practical HBM read ceiling the contraction kernels are set against."""
    import ctypes
    from paper_2508_21393_amd.build import PEAK_LIB
    if not os.path.exists(PEAK_LIB):
        return None
    L = ctypes.CDLL(PEAK_LIB)
    L.vlpeak_hbm_read_GBps.restype = ctypes.c_double
    L.vlpeak_hbm_read_GBps.argtypes = [ctypes.c_uint64]
    v = L.vlpeak_hbm_read_GBps(nbytes)
    return v if v > 0 else None


def serving_leg(B, n_requests, n_slots=8, seed=5, loads=(0.5, 0.8, 0.95), pool_n=14, planner=None):
    """Continuous batching at 13B-class shapes (hidden 5120, FFN 13824): a
    resident pool of proof requests that covers every target, T in
    {128, 512, 2048}, rank in {8, 16, 64} and type in {fwd, bwd, upd}
    (workloads.serving_sample), served by paper_2508_21393_amd.serve.  The
    saturated rate is measured first (the whole stream queued at once); then
    Poisson arrivals at each fraction of it in `loads`, n_requests each, each
    arrival proving a pooled witness with its own seed.  Three results per
    load are checked against a solo prove of the same request and seed.  The
    planner (if given) picks each pooled shape's launch shapes before the
    timed runs; the server uses its cached choices."""
    import numpy as np
    import torch
    import workloads
    from paper_2508_21393_amd import serve
    dev = lambda x: x if torch.is_tensor(x) else torch.from_numpy(x).to("cuda")  # noqa: E731
    weights, pool, shapes = {}, [], []
    for k, spec in enumerate(workloads.serving_sample(pool_n)):
        wl = workloads.serving_sample_workload(k, spec, weights, seed=seed, device="cuda")
        gas = [B.GroupArgs(g.group_id, [(dev(p.A), dev(p.B), p.transA, p.transB) for p in g.products], dev(g.C))
               for g in wl.groups]
        pool.append(gas)
        target, T, r, kind = spec
        shapes.append(f"{kind} {target} T={T} r={r}")
    torch.cuda.synchronize()
    planned = 0
    if planner is not None:
        for gas in pool:
            rec = planner.plan(gas, 1)
            planned += rec["lane_macs"] != 0
    solo = []
    for gas in pool:
        B.sumcheck_matmul_prove(gas, 1, mode=B.VL_MODE_BATCHED)
        t0 = time.perf_counter()
        B.sumcheck_matmul_prove(gas, 2, mode=B.VL_MODE_BATCHED)
        solo.append(time.perf_counter() - t0)
    mean_solo = sum(solo) / len(solo)
    rng = np.random.default_rng([seed, 11])
    picks = rng.integers(0, len(pool), size=n_requests)       # which pooled request each arrival proves
    srv = serve.ProofServer(n_slots=n_slots, hbm_budget_bytes=64 << 30, planner=planner)
    # warm the server (each slot's pinned buffers, the allocator's blocks):
    # every pooled request once per slot, back to back, not timed
    for i in range(n_slots * len(pool)):
        srv.submit(serve.Request(-1 - i, pool[i % len(pool)], 1))
    srv.drain()
    srv.done.clear()
    for slot in srv.slots:   # every slot's pinned buffers at the pool's largest request
        slot.host_buffers(torch, max(sum(B.proof_size(g) for g in gas) for gas in pool), max(len(gas) for gas in pool))
    n_products = sum(sum(len(g.prods) for g in pool[k]) for k in picks)
    gc.collect()
    gc.disable()   # no garbage-collector pass inside the timed loops
    rows = []
    try:
        # capacity: the whole stream queued at once (a standing backlog)
        _, sat_wall = serve.run_open_loop(srv, [(0.0, int(k)) for k in picks],
                                          lambda i, k: serve.Request(i, pool[k], 9000 + i))
        srv.done.clear()
        sat_rate = n_requests / sat_wall
        for li, frac in enumerate(loads):
            rate = frac * sat_rate
            gaps = np.random.default_rng([seed, 12, li]).exponential(1.0 / rate, size=n_requests)
            arrivals = [(float(t), int(k)) for t, k in zip(np.cumsum(gaps), picks)]
            base = 100000 * (li + 1)
            results, wall = serve.run_open_loop(srv, arrivals, lambda i, k: serve.Request(i, pool[k], base + i))
            srv.done.clear()
            gc.enable()
            for res in results[:: max(1, len(results) // 3)][:3]:
                ref, _ = B.sumcheck_matmul_prove(pool[arrivals[res.rid][1]], base + res.rid, mode=B.VL_MODE_BATCHED)
                assert res.proofs == ref and not any(res.status), "a served proof differs from the solo prove"
            gc.disable()
            summ = serve.latency_summary(results)
            worst = max(results, key=lambda r: r.latency)
            rows.append({"load": frac, "arrival_rate_per_s": rate, "requests": n_requests,
                         "p50_ms": summ["p50_ms"], "p99_ms": summ["p99_ms"], "mean_ms": summ["mean_ms"],
                         "requests_per_s": n_requests / wall, "products_per_s": n_products / wall,
                         "worst_request_ms": {"queued": 1e3 * (worst.t_admit - worst.t_arrive),
                                              "in_flight": 1e3 * (worst.t_done - worst.t_admit)},
                         "peak_in_flight": srv.peak_in_flight})
    finally:
        gc.enable()
    return {"workload": "13B-class LoRA layer requests (hidden 5120, FFN 13824; every target, T in "
                        "{128, 512, 2048}, rank in {8, 16, 64}, fwd/bwd/upd)",
            "pool": shapes, "slots": n_slots, "arrival": "poisson", "solo_mean_ms": 1e3 * mean_solo,
            "planned_shapes_off_default": planned,
            "saturated_requests_per_s": sat_rate, "saturated_products_per_s": n_products / sat_wall,
            "loads": rows}


def attention_leg(B, reps, seed=6):
    """Per-head batched products of one 7B-class attention layer (T = 2048,
    32 heads of 128): S = Q K^T, O = P V, dP = dO V^T, dV = P^T dO, dQ = dS K,
    dK = dS^T Q, proved in one vl_bmm_prove call (blocking) with the tensors
    resident in HBM.  Every proof is compared with the first call's bytes."""
    import torch
    import workloads
    layer = workloads.attention_layer(seed=seed, T=2048, H=32, dh=128, device="cuda")
    keep = []

    def dev(a):
        t = torch.from_numpy(a).to("cuda")
        keep.append(t)
        return t

    args = [B.BmmArgs(dev(hb.A.base), dev(hb.B.base), dev(hb.C.base), *hb.dims, hb.A.ld, hb.B.ld, hb.C.ld,
                      hb.A.head_stride, hb.B.head_stride, hb.C.head_stride, hb.transA, hb.transB, hb.group_id)
            for hb in layer]
    ws = torch.empty(B.bmm_workspace_size(args), dtype=torch.uint8, device="cuda")
    ref, _ = B.bmm_prove(args, seed, workspace=ws)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        pr, _ = B.bmm_prove(args, seed, workspace=ws)
        times.append(time.perf_counter() - t0)
        assert pr == ref, "attention proofs changed between calls"
    ms = 1e3 * sorted(times)[len(times) // 2]
    macs = sum(H * (d0 * d1 + d1 * d2 + d0 * d2) for (H, d0, d1, d2) in (hb.dims for hb in layer))
    nbytes = sum(hb.A.base.nbytes + hb.B.base.nbytes + hb.C.base.nbytes for hb in layer)
    return {"workload": "7B-class attention layer, T=2048, 32 heads x 128: S=QK^T, O=PV, dP=dOV^T, dV=P^TdO, "
                        "dQ=dSK, dK=dS^TQ (per-head batched sumchecks, one call)",
            "products": len(layer), "heads": 32, "ms_per_call": ms, "calls": reps,
            "Fr_MAC_per_s": macs / (ms * 1e-3), "algorithmic_macs": macs,
            "operand_bytes": nbytes, "operand_GBps": nbytes / (ms * 1e-3) / 1e9}


def lookup_leg(B, reps, seed=61):
    """Lookup arguments at 7B-class size: a range check of 2^23 int16
    activations (T = 2048 x hidden 4096) against the int16 table (2^16 rows)
    and the SiLU input/output check of 2^23 entries against its 2^16-row
    table, proved in one vl_lookup_prove call (blocking)."""
    import torch
    import workloads
    cases = [workloads.lookup_range(73, 1 << 23, 0), workloads.lookup_silu(74, 1 << 23, 1)]
    keep = []

    def dev(a):
        if a is None:
            return None
        t = torch.from_numpy(a).to("cuda")
        keep.append(t)
        return t

    args = [B.LookupArgs(dev(c.x), dev(c.y), dev(c.tb), c.t0, c.N, len(c.x), c.x.dtype, c.y is not None, c.lid,
                         dtype_y=c.y.dtype if c.y is not None else None) for c in cases]
    ws = torch.empty(B.lookup_workspace_size(args), dtype=torch.uint8, device="cuda")
    ref, _ = B.lookup_prove(args, seed, workspace=ws)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        pr, _ = B.lookup_prove(args, seed, workspace=ws)
        times.append(time.perf_counter() - t0)
        assert pr == ref, "lookup proofs changed between calls"
    ms = 1e3 * sorted(times)[len(times) // 2]
    entries = sum(len(c.x) for c in cases)
    return {"workload": "lookup arguments, 7B-class: range check of 2^23 int16 activations and SiLU "
                        "input/output check of 2^23 entries, tables of 2^16 rows (one call)",
            "lookups": len(cases), "entries": entries, "ms_per_call": ms, "calls": reps,
            "entries_per_s": entries / (ms * 1e-3)}


def hyrax_leg(B, reps, seed=4, hidden=4096, ffn=11008):
    """Hyrax commitments to the frozen weights of one 7B-class block (W_q,
    W_k, W_v, W_o 4096 x 4096, W_gate, W_up 4096 x 11008, W_down 11008 x
    4096; int16), one row commitment per matrix row, with a fixed-base table
    of 11008 generators (set up once, timed separately).  Each rep commits
    the seven matrices back to back on one stream, timed with HIP events;
    one opening of W_q at a random point is checked by the host verifier.
    Algorithmic work: one mixed addition per nonzero signed base-256 digit of
    the entries, 10 Montgomery products of 12 x 12 32-bit limbs each, i.e.
    2880 32 x 32 -> 64-bit multiply-adds; peak: 256 CUs x 64 lanes x 2.4 GHz
    = 39.3 T such multiply-adds/s (v_mad_u64_u32 issues at full rate)."""
    import random
    import numpy as np
    import torch
    import workloads
    mats = workloads.block_weights(seed=seed, hidden=hidden, ffn=ffn)
    m_max = max(W.shape[1] for _, W in mats)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    table = B.HyraxTable(m_max, 2)
    ev[1].record()
    torch.cuda.synchronize()
    setup_ms = ev[0].elapsed_time(ev[1])
    devs, outs, wss, nz = [], [], [], 0
    for _, W in mats:
        Wd = torch.from_numpy(W).cuda()
        R, m = W.shape
        devs.append(Wd)
        outs.append(torch.empty((R, B.HYRAX_POINT_BYTES), dtype=torch.uint8, device="cuda"))
        wss.append(torch.empty(max(256, B.hyrax_commit_workspace_size(R, m)), dtype=torch.uint8, device="cuda"))
        v = W.astype(np.int64)
        d0 = ((v + 128) & 255) - 128
        nz += int(np.count_nonzero(d0)) + int(np.count_nonzero((v - d0) >> 8))
    for Wd, o, ws in zip(devs, outs, wss):
        B.hyrax_commit(Wd, table, out=o, workspace=ws)
    torch.cuda.synchronize()
    ref = [o.cpu() for o in outs]
    # per matrix on one stream (its own time); then the block with the
    # matrices alternating between two streams, so that one matrix's final
    # kernel (one inversion per 64 rows, a few waves) overlaps the next one's
    # commit kernel
    per = [[] for _ in mats]
    totals = []
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(len(mats) + 1)]
    for _ in range(reps):
        evs[0].record()
        for k, (Wd, o, ws) in enumerate(zip(devs, outs, wss)):
            B.hyrax_commit(Wd, table, out=o, workspace=ws)
            evs[k + 1].record()
        torch.cuda.synchronize()
        for k in range(len(mats)):
            per[k].append(evs[k].elapsed_time(evs[k + 1]))
    streams = [torch.cuda.current_stream(), torch.cuda.Stream()]
    e_start, e_end, e_side = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
                              torch.cuda.Event())
    for _ in range(reps):
        e_start.record(streams[0])
        streams[1].wait_event(e_start)
        for k, (Wd, o, ws) in enumerate(zip(devs, outs, wss)):
            B.hyrax_commit(Wd, table, out=o, workspace=ws, stream=streams[k % 2])
        e_side.record(streams[1])
        streams[0].wait_event(e_side)
        e_end.record(streams[0])
        torch.cuda.synchronize()
        totals.append(e_start.elapsed_time(e_end))
    for o, r in zip(outs, ref):
        assert torch.equal(o.cpu(), r), "commitments changed between calls"
    ms = sorted(totals)[len(totals) // 2]
    entries = sum(W.size for _, W in mats)
    # one opening of W_q, checked on the host
    (_, Wq), Cq = mats[0], ref[0].numpy().tobytes()
    rng = random.Random(seed)
    p_mod = B.FR_MODULUS
    x = [rng.randrange(p_mod) for _ in range(nv(Wq.shape[0]))]
    y = [rng.randrange(p_mod) for _ in range(nv(Wq.shape[1]))]
    t0 = time.perf_counter()
    w = B.hyrax_open(devs[0], x)
    t_open = time.perf_counter() - t0
    t0 = time.perf_counter()
    ok, _, msg = B.hyrax_verify_open(Cq, Wq.shape[0], Wq.shape[1], x, y, w)
    t_ver = time.perf_counter() - t0
    assert ok, msg
    madd_per_s = nz / (ms * 1e-3)
    peak_t = 256 * 64 * 2.4e9 / 1e12
    achieved_t = madd_per_s * 2880 / 1e12
    return {"workload": "Hyrax row commitments to the frozen int16 weights of one 7B-class block "
                        "(q, k, v, o 4096x4096; gate, up 4096x11008; down 11008x4096), table of 11008 generators",
            "matrices": len(mats), "entries": entries, "commitments": sum(W.shape[0] for _, W in mats),
            "commitment_bytes": 96 * sum(W.shape[0] for _, W in mats),
            "setup_ms": setup_ms, "ms_per_block": ms, "reps": reps, "streams": 2,
            "ms_per_matrix": {name: sorted(t)[len(t) // 2] for (name, _), t in zip(mats, per)},
            "entries_per_s": entries / (ms * 1e-3), "mixed_additions": nz, "mixed_additions_per_s": madd_per_s,
            "open_ms_wq": 1e3 * t_open, "verify_open_ms_wq": 1e3 * t_ver,
            "roofline": {"bound": "alu", "achieved": achieved_t, "peak": peak_t,
                         "unit": "T 32x32->64-bit multiply-adds/s (2880 per mixed addition)",
                         "frac": achieved_t / peak_t,
                         "note": "block time on two streams (commit and final kernels of consecutive "
                                 "matrices overlap)"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--T", type=int, default=2048)
    ap.add_argument("--mode", default="batched", choices=["batched", "per_instance", "persistent"])
    ap.add_argument("--per-instance-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-peak", action="store_true")
    ap.add_argument("--lane-macs", type=int, default=0, help="vl_tuning.lane_macs (0: library default)")
    ap.add_argument("--min-tasks", type=int, default=0, help="vl_tuning.min_tasks (0: library default)")
    ap.add_argument("--contract-streams", type=int, default=0,
                    help="vl_tuning.contract_streams (0: library default; 1: one stream; 2: two)")
    ap.add_argument("--segments", type=int, default=0, help="vl_tuning.segments (0: library default)")
    ap.add_argument("--cols-rows", type=int, default=0, help="vl_tuning.cols_rows (0: library default)")
    ap.add_argument("--claim-order", type=int, default=0,
                    help="vl_tuning.claim_order (0: library default, 1: C by columns, 2: C by rows)")
    ap.add_argument("--inflight", type=int, default=8,
                    help="proofs in flight in the throughput phase (asynchronous entry point)")
    ap.add_argument("--graph", type=int, default=1,
                    help="1: the throughput phase replays one captured HIP graph per slot (vl_prove_graph)")
    ap.add_argument("--serve-slots", type=int, default=8, help="slots of the serving leg's proof server")
    ap.add_argument("--serve-requests", type=int, default=600,
                    help="requests per offered load in the serving leg at 13B-class shapes (0: skip it)")
    ap.add_argument("--no-plan", action="store_true",
                    help="use the library's default launch shapes instead of the planner's choice")
    ap.add_argument("--plan-cache", default=None,
                    help="JSON file of the planner's choices per shape signature (read and updated)")
    ap.add_argument("--attention-reps", type=int, default=5,
                    help="calls of the attention-layer leg (per-head batched products; 0: skip it)")
    ap.add_argument("--lookup-reps", type=int, default=3,
                    help="calls of the lookup-argument leg (0: skip it)")
    ap.add_argument("--hyrax-reps", type=int, default=3,
                    help="repetitions of the Hyrax commitment leg (0 skips it)")
    ap.add_argument("--legs-only", action="store_true",
                    help="run only the attention, lookup and Hyrax legs (for profiling them)")
    args = ap.parse_args()
    ws = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or ws != 1:
        print("bench.py measures one GPU: the prover's groups are independent (each has its own "
              "transcript), so a multi-GPU prover would shard the groups across GPUs; this benchmark "
              "runs on a single MI355X: run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_2508_21393_amd import binding as B

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    B.lib()
    mode = {"batched": B.VL_MODE_BATCHED, "per_instance": B.VL_MODE_PER_INSTANCE,
            "persistent": B.VL_MODE_PERSISTENT}[args.mode]
    if args.legs_only:
        legs = {}
        if args.attention_reps > 0:
            legs["attention"] = attention_leg(B, args.attention_reps)
            torch.cuda.empty_cache()
        if args.lookup_reps > 0:
            legs["lookup"] = lookup_leg(B, args.lookup_reps)
            torch.cuda.empty_cache()
        if args.hyrax_reps > 0:
            legs["hyrax"] = hyrax_leg(B, args.hyrax_reps)
        print(json.dumps(legs), flush=True)
        return
    t_gen = time.perf_counter()
    w = workloads.config4(T=args.T, device="cuda")
    groups = w.groups
    dev = lambda x: torch.from_numpy(x).to("cuda")  # noqa: E731
    gas = [B.GroupArgs(g.group_id, [(dev(p.A), dev(p.B), p.transA, p.transB) for p in g.products],
                       dev(g.C)) for g in groups]
    batch = B.GroupBatch(gas)   # the vl_group array, built once for every call
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    shapes = [g.shapes for g in groups]
    macs = algorithmic_macs(shapes)
    n_products = sum(len(s) for s in shapes)
    tun = B.tuning(args.lane_macs, args.min_tasks, args.segments, args.cols_rows, 0, args.claim_order,
                   args.contract_streams)
    from paper_2508_21393_amd import tune
    planner = None if args.no_plan else tune.Planner(cache_path=args.plan_cache)
    plan_rec = None
    knobs = (args.lane_macs, args.min_tasks, args.segments, args.cols_rows, args.claim_order, args.contract_streams)
    if planner is not None and not any(knobs) and mode == B.VL_MODE_BATCHED:
        plan_rec = planner.plan(batch, w.seed, mode)
        tun = planner.tuning(batch, w.seed, mode)
    one_seg = B.tuning(tun.lane_macs, tun.min_tasks, tun.segments or 1, tun.cols_rows, 0, tun.claim_order,
                       tun.contract_streams)
    workspace = torch.empty(max(B.workspace_size(batch, mode, tuning_=tun),
                                B.workspace_size(batch, mode, tuning_=one_seg)), dtype=torch.uint8, device="cuda")

    def step(stage=None, tuning_=None):
        return B.sumcheck_matmul_prove(batch, w.seed, mode=mode, workspace=workspace, stage_ms=stage,
                                       tuning_=tuning_ or tun)

    for _ in range(args.warmup):
        ref, ref_dig = step()
    torch.cuda.synchronize()
    ref_cat = b"".join(ref)

    # Throughput: `inflight` proofs in flight, each on its own stream with
    # its own workspace (a captured prove graph per slot, replayed per proof,
    # or the asynchronous entry point with --graph 0); the host plans the
    # next proof while the GPU runs earlier ones, and one proof's single-CU
    # sumcheck rounds overlap the next one's contractions.  The kernels write
    # each proof straight into pinned host memory (a copy-engine transfer
    # per proof would order the streams behind each other); every proof is
    # compared with the reference bytes.
    n_groups = len(groups)

    class Slot:
        def __init__(self):
            self.stream = torch.cuda.Stream()
            self.ws = torch.empty(max(256, B.workspace_size(batch, mode, async_=True, tuning_=tun)),
                                  dtype=torch.uint8, device="cuda")
            self.proofs = torch.empty(batch.total, dtype=torch.uint8, pin_memory=True)
            self.status = torch.empty(n_groups, dtype=torch.int32, pin_memory=True)
            self.done = torch.cuda.Event()
            self.pending = False
            self.graph = B.ProveGraph(batch, self.ws, self.proofs, self.status, tuning_=tun) if args.graph else None

        def submit(self):
            if self.graph is not None:
                self.graph.launch(w.seed, stream=self.stream)
            else:
                B.sumcheck_matmul_prove_async(batch, w.seed, self.proofs, self.status, self.ws, mode=mode,
                                              stream=self.stream, tuning_=tun)
            self.done.record(self.stream)
            self.pending = True

        def collect(self):
            # numpy views of the pinned buffers: a torch CPU op here would
            # wake torch's thread pool, whose spinning threads then hold up
            # the prover's host-side hashing threads of the next submit
            self.done.synchronize()
            st, pr = self.status.numpy(), self.proofs.numpy()
            assert not st.any(), "a group failed"
            assert pr.tobytes() == ref_cat, "proofs differ from the blocking run"
            pr[:] = 0
            self.pending = False

    slots = [Slot() for _ in range(max(1, args.inflight))]

    def pipelined(nsteps):
        for i in range(nsteps):
            sl = slots[i % len(slots)]
            if sl.pending:
                sl.collect()
            sl.submit()
        for sl in slots:
            if sl.pending:
                sl.collect()

    pipelined(max(args.warmup, len(slots)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pipelined(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps

    # Latency: one proof at a time through the blocking entry point, host
    # clock around each call
    lat = []
    tb = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        proofs, dig = step()
        lat.append(time.perf_counter() - s0)
        assert dig == ref_dig, "proofs changed between steps"
    torch.cuda.synchronize()
    blocking_ms = 1e3 * (time.perf_counter() - tb) / args.steps
    lat_ms = sorted(1e3 * x for x in lat)
    p50 = lat_ms[len(lat_ms) // 2]
    p99 = lat_ms[min(len(lat_ms) - 1, int(math.ceil(0.99 * len(lat_ms))) - 1)]
    # Stage times: blocking calls with HIP events around every launch (the
    # events add host work per launch, so these calls are not the ones timed
    # for latency), in one pipeline segment (unless one was asked for) so
    # that each contraction kind is one launch per proof, whose time is the
    # kernel's own (the library runs them on one stream when stage times are
    # asked for)
    stage_tun = one_seg
    stage_sum, ilat = [0.0] * B.VL_STAGE_COUNT, []
    for _ in range(args.steps):
        s0 = time.perf_counter()
        st = []
        proofs, dig = step(st, stage_tun)
        ilat.append(time.perf_counter() - s0)
        stage_sum = [a + b for a, b in zip(stage_sum, st)]
        assert dig == ref_dig, "proofs changed between steps"
    stage_avg = [x / args.steps for x in stage_sum]
    instrumented_p50 = sorted(1e3 * x for x in ilat)[len(ilat) // 2]

    # per-instance prover on the same inputs (the baseline the batched path must beat)
    per_inst_ms = None
    if mode != B.VL_MODE_PER_INSTANCE and args.per_instance_steps > 0:
        ws_pi = torch.empty(B.workspace_size(batch, B.VL_MODE_PER_INSTANCE), dtype=torch.uint8, device="cuda")
        pi, _ = B.sumcheck_matmul_prove(batch, w.seed, mode=B.VL_MODE_PER_INSTANCE, workspace=ws_pi)
        assert pi == ref, "per-instance proofs differ from the batched ones"
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.per_instance_steps):
            B.sumcheck_matmul_prove(batch, w.seed, mode=B.VL_MODE_PER_INSTANCE, workspace=ws_pi)
        torch.cuda.synchronize()
        per_inst_ms = 1e3 * (time.perf_counter() - t1) / args.per_instance_steps
        del ws_pi

    # dominant kernel: the contraction kind with the most device time.  Its
    # algorithmic traffic is the matrix bytes it must stream (every entry
    # once); the eq digits and partial sums are small and mostly cache hits.
    kinds = contraction_bytes(groups, cols_rows=tun.cols_rows, claim_order=tun.claim_order)
    dom = max(kinds, key=lambda k: stage_avg[k])
    dom_ms = stage_avg[dom]
    dom_bytes, dom_entries = kinds[dom]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9 if dom_ms > 0 else 0.0
    rates = None if args.no_peak else peak_rates()
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_GBPS, "unit": "GB/s",
                "frac": achieved / HBM_GBPS, "traffic": measured_traffic(B.STAGE_NAMES[dom]),
                "kernel": f"contract_kernel {B.STAGE_NAMES[dom]} (eq digits x matrix digits, v_mad_i64_i32)",
                "bytes_per_launch": dom_bytes, "entries_per_launch": dom_entries, "avg_launch_ms": dom_ms,
                "per_kind": {B.STAGE_NAMES[k]: {"ms": stage_avg[k], "GBps": b / (stage_avg[k] * 1e-3) / 1e9
                                                if stage_avg[k] > 0 else None,
                                                "valu_frac": (e * MAD_PER_ENTRY[B.STAGE_NAMES[k]] /
                                                              (stage_avg[k] * 1e-3) / (CU * LANES_PER_CLK * CLOCK_HZ))
                                                if stage_avg[k] > 0 else None,
                                                "traffic_ratio": (measured_traffic(B.STAGE_NAMES[k]) / b
                                                                  if measured_traffic(B.STAGE_NAMES[k]) else None)}
                             for k, (b, e) in kinds.items()}}
    if not args.no_peak:
        rd = streaming_read_GBps()
        roofline["streaming_read_GBps"] = rd
        roofline["frac_of_streaming_read"] = achieved / rd if rd else None

    out = {
        "metric": METRIC, "value": macs * args.steps / elapsed, "unit": "Fr-MAC/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "Fr (BLS12-381 scalar field, exact); int16 operands, int64 outputs",
        "data": "synthetic (seeded int16 fixed-point tensors, no model weights or dataset)",
        "config": {"workload": f"7B-class block T={args.T}, hidden 4096, FFN 11008, LoRA r16 on "
                               f"q,k,v,o,gate,up,down: fwd+bwd+update", "groups": len(groups),
                   "products": n_products, "mode": args.mode, "algorithmic_macs_per_step": macs},
        "proofs_per_s": n_products * args.steps / elapsed,
        "latency_ms": {"p50": p50, "p99": p99, "blocking_ms_per_step": blocking_ms,
                       "p50_with_stage_events": instrumented_p50},
        "inflight": len(slots),
        "graph": bool(args.graph),
        "per_instance_ms_per_step": per_inst_ms,
        "speedup_vs_per_instance": (per_inst_ms / ms_per_step) if per_inst_ms else None,
        "speedup_vs_per_instance_blocking": (per_inst_ms / blocking_ms) if per_inst_ms else None,
        "stage_ms": {B.STAGE_NAMES[i]: stage_avg[i] for i in range(B.VL_STAGE_COUNT) if stage_avg[i] > 0},
        "roofline": roofline,
        "valu_lane_ops_per_s": rates,
        "witness_setup_s": t_gen,
        "tuning": {"lane_macs": tun.lane_macs, "min_tasks": tun.min_tasks, "segments": tun.segments,
                   "cols_rows": tun.cols_rows, "claim_order": tun.claim_order,
                   "contract_streams": tun.contract_streams},
    }
    if plan_rec is not None:
        out["plan"] = {"signature": tune.signature(batch, mode),
                       "chosen": {k: plan_rec[k] for k in ("lane_macs", "segments", "cols_rows", "claim_order")},
                       "blocking_ms_chosen": plan_rec["ms"], "blocking_ms_default": plan_rec["default_ms"],
                       "candidates": len(plan_rec["grid"]),
                       "note": "0 = the library default for that knob; timed on this block's inputs"}
    if args.serve_requests > 0:
        for sl in slots:
            sl.graph = None
        del slots, workspace, batch, gas
        torch.cuda.empty_cache()
        out["serving"] = serving_leg(B, args.serve_requests, n_slots=args.serve_slots, planner=planner)
    if args.attention_reps > 0:
        torch.cuda.empty_cache()
        out["attention"] = attention_leg(B, args.attention_reps)
    if args.lookup_reps > 0:
        torch.cuda.empty_cache()
        out["lookup"] = lookup_leg(B, args.lookup_reps)
    if args.hyrax_reps > 0:
        torch.cuda.empty_cache()
        out["hyrax"] = hyrax_leg(B, args.hyrax_reps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
