"""Write the stored expected proofs under tests/golden/ by running the CPU oracle.

Only ``oracle`` and ``workloads`` are used: every stored value is what the
oracle computes for the seeded synthetic inputs.  Usage:

    python tests/golden/make_golden.py [cfg1 cfg1_sweep tiny cfg2 cfg3 cfg4 cfg5 chain bmm lookup lookup_full] [--procs N]

Each config file lists, per group: name, group id, shapes, the SHA-256 of the
proof bytes and the final transcript state; small configs also keep the full
proof in hex.  cfg5 lists the requests of the 13B-class serving sample
(workloads.serving_sample), each with its seed and its groups.  bmm lists
the per-head batched products (oracle/bmm.py).
"""
import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle.zkmat import prove_workload_group  # noqa: E402
import workloads  # noqa: E402

_W = None


def _prove(i):
    g = _W.groups[i]
    t = time.time()
    proof, state, det = prove_workload_group(g, _W.seed)
    return i, proof, state, time.time() - t


def record(w, keep_hex: bool, procs: int):
    global _W
    _W = w
    idx = list(range(len(w.groups)))
    # largest groups first so the pool's tail is short
    idx.sort(key=lambda i: -sum(d0 * d1 + d1 * d2 for d0, d1, d2 in w.groups[i].shapes))
    if procs > 1:
        with mp.get_context("fork").Pool(procs) as pool:
            res = pool.map(_prove, idx, chunksize=1)
    else:
        res = [_prove(i) for i in idx]
    res.sort()
    out = []
    for i, proof, state, dt in res:
        g = w.groups[i]
        e = dict(name=g.name, group_id=g.group_id, shapes=[list(s) for s in g.shapes],
                 proof_sha256=hashlib.sha256(proof).hexdigest(), state=state.hex(),
                 proof_len=len(proof))
        if keep_hex:
            e["proof_hex"] = proof.hex()
        out.append(e)
        print(f"  {g.name:28s} {g.shapes} {dt:7.1f}s", flush=True)
    return dict(workload=w.name, seed=w.seed, groups=out)


TINY = [
    # (seed, dims list, dtype, trans, value_bits)
    (11, [(1, 1, 1)], "int16", (False, False), None),
    (12, [(3, 5, 7)], "int16", (False, False), None),
    (13, [(5, 1, 3)], "int16", (True, False), None),
    (14, [(1, 300, 1)], "int16", (False, True), None),
    (15, [(70, 33, 130)], "int16", (True, True), None),
    (16, [(17, 64, 9), (17, 3, 9)], "int16", (False, True), None),
    (17, [(40, 257, 65)], "int32", (False, False), 20),
    (18, [(33, 19, 47)], "int64", (True, False), 24),
    (19, [(300, 520, 129)], "int16", (False, False), None),
]


def tiny_groups():
    import numpy as np
    out = []
    for k, (seed, dims, dt, trans, vb) in enumerate(TINY):
        g = workloads.tiny_random_group(seed, dims, dtype=getattr(np, dt), trans=trans,
                                        value_bits=vb, name=f"tiny{k}")
        g.group_id = k
        out.append(g)
    return workloads.Workload("tiny parity cases", 1234, out)


N_CFG5 = 14   # requests of the 13B-class serving sample (workloads.serving_sample)

_JOBS = None


def _prove_job(i):
    w, gi = _JOBS[i]
    g = w.groups[gi]
    t = time.time()
    proof, state, _ = prove_workload_group(g, w.seed)
    return i, proof, state, time.time() - t


def record_cfg5(procs: int):
    """The serving sample at 13B-class shapes: every group of every request,
    proved by the oracle with the request's own seed."""
    global _JOBS
    specs = workloads.serving_sample(N_CFG5)
    weights = {}
    reqs = [workloads.serving_sample_workload(k, sp, weights) for k, sp in enumerate(specs)]
    _JOBS = [(w, gi) for w in reqs for gi in range(len(w.groups))]
    idx = sorted(range(len(_JOBS)), key=lambda i: -sum(d0 * d1 + d1 * d2 + d0 * d2 for d0, d1, d2 in
                                                        _JOBS[i][0].groups[_JOBS[i][1]].shapes))
    if procs > 1:
        with mp.get_context("fork").Pool(procs) as pool:
            res = pool.map(_prove_job, idx, chunksize=1)
    else:
        res = [_prove_job(i) for i in idx]
    by_job = {i: (proof, state, dt) for i, proof, state, dt in res}
    out, j = [], 0
    for k, (sp, w) in enumerate(zip(specs, reqs)):
        groups = []
        for g in w.groups:
            proof, state, dt = by_job[j]
            j += 1
            groups.append(dict(name=g.name, group_id=g.group_id, shapes=[list(x) for x in g.shapes],
                               proof_sha256=hashlib.sha256(proof).hexdigest(), state=state.hex(),
                               proof_len=len(proof)))
            print(f"  req{k:<2d} {g.name:34s} {g.shapes} {dt:7.1f}s", flush=True)
        out.append(dict(request=k, target=sp[0], T=sp[1], rank=sp[2], kind=sp[3], seed=w.seed,
                        workload=w.name, groups=groups))
    return dict(workload="13B-class serving sample (hidden 5120, FFN 13824)", n=N_CFG5, requests=out)


CHAIN_TINY = [
    # (seed, T, d_in, d_out, r): shapes with ragged and unit dimensions
    (21, 8, 12, 10, 3), (22, 4, 4, 4, 2), (23, 5, 7, 9, 1), (24, 1, 3, 2, 2), (25, 16, 8, 32, 4),
    (26, 3, 1, 5, 1), (27, 70, 130, 33, 16), (28, 64, 256, 300, 8),
]
CHAIN_SEED = 31


def record_chain():
    """Chained layer proofs (oracle/chain.py): the tiny layers in full and
    the FFN-up layer of the backward-and-update configuration by digest."""
    from oracle.chain import chain_prove
    tiny = []
    for seed, T, d_in, d_out, r in CHAIN_TINY:
        w = workloads.tiny_layer(seed, T, d_in, d_out, r)
        t = time.time()
        proof, state, _ = chain_prove(w, CHAIN_SEED)
        tiny.append(dict(spec=[seed, T, d_in, d_out, r], proof_hex=proof.hex(), state=state.hex()))
        print(f"  tiny layer {(T, d_in, d_out, r)} {time.time() - t:6.1f}s", flush=True)
    w = workloads.chain_layer()
    t = time.time()
    proof, state, _ = chain_prove(w, CHAIN_SEED)
    print(f"  layer {w.dims} {time.time() - t:6.1f}s", flush=True)
    full = dict(dims=list(w.dims), proof_sha256=hashlib.sha256(proof).hexdigest(), state=state.hex(),
                proof_len=len(proof))
    return dict(seed=CHAIN_SEED, F=w.F, eta=w.eta, tiny=tiny, layer=full)


BMM_TINY = [
    # (seed, H, D0, D1, D2, options of workloads.tiny_head_batch)
    (41, 1, 1, 1, 1, {}),
    (42, 3, 5, 7, 6, dict(transA=True, b_cols=True, c_cols=True)),
    (43, 2, 3, 1, 5, dict(a_cols=True)),
    (44, 5, 1, 4, 1, dict(transB=True)),
    (45, 8, 2, 2, 4, dict(transA=True, transB=True, a_cols=True, b_cols=True)),
    (46, 3, 70, 33, 130, dict(c_cols=True)),
    (47, 6, 40, 257, 65, dict(transA=True)),
    (48, 32, 64, 16, 64, dict(a_cols=True, b_cols=True, transB=True)),
    (49, 4, 300, 129, 20, dict(b_cols=True, c_cols=True)),
    # tables of 2^14 .. 2^15 entries: the first rounds run GPU-wide
    (50, 8, 3, 2048, 5, dict(b_cols=True)),
    (51, 2, 2, 16384, 3, dict(transA=True)),
    (52, 1, 4, 20000, 2, {}),
]
ATTN_SMALL = dict(seed=7, T=256, H=4, dh=32)
ATTN_FULL = dict(seed=6, T=2048, H=32, dh=128)
BMM_SEED = 41

_BATCHES = None


def _prove_batch(i):
    from oracle.bmm import prove_batch
    t = time.time()
    proof, state, _ = prove_batch(_BATCHES[i], BMM_SEED)
    return i, proof, state, time.time() - t


def _bmm_records(batches, keep_hex, procs):
    global _BATCHES
    _BATCHES = batches
    idx = list(range(len(batches)))
    if procs > 1:
        with mp.get_context("fork").Pool(min(procs, len(idx))) as pool:
            res = pool.map(_prove_batch, idx, chunksize=1)
    else:
        res = [_prove_batch(i) for i in idx]
    out = []
    for i, proof, state, dt in sorted(res):
        b = batches[i]
        e = dict(name=b.name, group_id=b.group_id, dims=list(b.dims), proof_sha256=hashlib.sha256(proof).hexdigest(),
                 state=state.hex(), proof_len=len(proof))
        if keep_hex:
            e["proof_hex"] = proof.hex()
        out.append(e)
        print(f"  {b.name:12s} {b.dims} {dt:7.1f}s", flush=True)
    return out


def record_bmm(procs: int):
    """Per-head batched products (oracle/bmm.py): the tiny cases and a small
    attention layer in full, the 7B-class attention layer (T = 2048, 32 heads
    of 128) by digest."""
    tiny = []
    for k, (seed, H, d0, d1, d2, kw) in enumerate(BMM_TINY):
        b = workloads.tiny_head_batch(seed, H, d0, d1, d2, name=f"bmm{k}", **kw)
        b.group_id = k
        tiny.append(b)
    data = dict(seed=BMM_SEED, tiny_spec=[[s, H, d0, d1, d2, kw] for s, H, d0, d1, d2, kw in BMM_TINY],
                tiny=_bmm_records(tiny, True, procs))
    data["attn_small_spec"] = ATTN_SMALL
    data["attn_small"] = _bmm_records(workloads.attention_layer(**ATTN_SMALL), True, procs)
    data["attn_full_spec"] = ATTN_FULL
    data["attn_full"] = _bmm_records(workloads.attention_layer(**ATTN_FULL), False, procs)
    return data


LOOKUP_TINY = [
    # (seed, D, N, t0, two_col)
    (61, 20, 8, -3, True), (62, 8, 8, 5, False), (63, 64, 4, 0, False), (64, 3, 16, -100, True),
    (65, 37, 2, 7, False), (66, 1, 1, 2, False), (67, 5000, 64, -32, True), (68, 20000, 16, 1000, False),
    (69, 9000, 16384, -8192, True),
]
LOOKUP_MID = [("range", 71, 1 << 16), ("silu", 72, 1 << 18)]
LOOKUP_FULL = [("range", 73, 1 << 23), ("silu", 74, 1 << 23)]
LOOKUP_SEED = 61

_LOOKUPS = None


def _prove_lookup(i):
    from oracle.lookup import prove_case
    t = time.time()
    proof, state, _ = prove_case(_LOOKUPS[i], LOOKUP_SEED)
    return i, proof, state, time.time() - t


def _lookup_records(cases, keep_hex, procs):
    global _LOOKUPS
    _LOOKUPS = cases
    idx = sorted(range(len(cases)), key=lambda i: -len(cases[i].x))
    if procs > 1:
        with mp.get_context("fork").Pool(min(procs, len(idx))) as pool:
            res = pool.map(_prove_lookup, idx, chunksize=1)
    else:
        res = [_prove_lookup(i) for i in idx]
    out = []
    for i, proof, state, dt in sorted(res):
        c = cases[i]
        e = dict(name=c.name, D=len(c.x), N=c.N, proof_sha256=hashlib.sha256(proof).hexdigest(), state=state.hex(),
                 proof_len=len(proof))
        if keep_hex:
            e["proof_hex"] = proof.hex()
        out.append(e)
        print(f"  {c.name:24s} {dt:7.1f}s", flush=True)
    return out


def _lookup_case(kind, seed, D, lid):
    return (workloads.lookup_range if kind == "range" else workloads.lookup_silu)(seed, D, lid)


def record_lookup(procs: int, full: bool):
    """Lookup arguments (oracle/lookup.py): tiny cases in full, two
    mid-size cases (a range check of 2^16 activations, the SiLU input/output
    check of 2^18) in full, and with ``full`` the 7B-class cases (2^23
    activations: range check and SiLU check) by digest."""
    tiny = [workloads.tiny_lookup(s, D, N, t0, two, lid=k) for k, (s, D, N, t0, two) in enumerate(LOOKUP_TINY)]
    data = dict(seed=LOOKUP_SEED, tiny_spec=LOOKUP_TINY, tiny=_lookup_records(tiny, True, procs))
    mid = [_lookup_case(kind, s, D, k) for k, (kind, s, D) in enumerate(LOOKUP_MID)]
    data["mid_spec"] = LOOKUP_MID
    data["mid"] = _lookup_records(mid, True, procs)
    if full:
        big = [_lookup_case(kind, s, D, k) for k, (kind, s, D) in enumerate(LOOKUP_FULL)]
        data["full_spec"] = LOOKUP_FULL
        data["full"] = _lookup_records(big, False, procs)
    return data


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("configs", nargs="*", default=["cfg1", "tiny", "cfg2", "cfg3"])
    ap.add_argument("--procs", type=int, default=os.cpu_count())
    args = ap.parse_args()
    for name in args.configs:
        t = time.time()
        print(f"{name}: generating", flush=True)
        if name == "chain":
            data = record_chain()
            with open(os.path.join(HERE, "chain.json"), "w") as f:
                json.dump(data, f, indent=1)
            print(f"{name}: done in {time.time() - t:.1f}s", flush=True)
            continue
        if name in ("lookup", "lookup_full"):
            path = os.path.join(HERE, "lookup.json")
            data = record_lookup(args.procs, name == "lookup_full")
            if name == "lookup" and os.path.exists(path):
                old = json.load(open(path))
                if "full" in old:
                    data["full_spec"], data["full"] = old["full_spec"], old["full"]
            with open(path, "w") as f:
                json.dump(data, f, indent=1)
            print(f"{name}: done in {time.time() - t:.1f}s", flush=True)
            continue
        if name == "bmm":
            data = record_bmm(args.procs)
            with open(os.path.join(HERE, "bmm.json"), "w") as f:
                json.dump(data, f, indent=1)
            print(f"{name}: done in {time.time() - t:.1f}s", flush=True)
            continue
        if name == "cfg5":
            data = record_cfg5(args.procs)
            with open(os.path.join(HERE, "cfg5.json"), "w") as f:
                json.dump(data, f, indent=1)
            print(f"{name}: done in {time.time() - t:.1f}s", flush=True)
            continue
        if name == "tiny":
            w = tiny_groups()
        elif name == "cfg1_sweep":
            data = [record(workloads.config1(seed=s), True, 1) for s in range(1, 17)]
            with open(os.path.join(HERE, "cfg1_sweep.json"), "w") as f:
                json.dump(data, f, indent=1)
            continue
        else:
            w = workloads.make_config(name)
        print(f"{name}: proving {len(w.groups)} groups", flush=True)
        data = record(w, keep_hex=name in ("cfg1", "tiny"), procs=args.procs)
        data["tiny_spec"] = TINY if name == "tiny" else None
        with open(os.path.join(HERE, f"{name}.json"), "w") as f:
            json.dump(data, f, indent=1)
        print(f"{name}: done in {time.time() - t:.1f}s", flush=True)


if __name__ == "__main__":
    main()
