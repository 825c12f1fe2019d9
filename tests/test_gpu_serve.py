"""Continuous-batching server: each result is the oracle's proof, alone and in the mix.

Every served proof is compared with the CPU oracle's bytes for the same
request (tiny shapes here, proved by the oracle in milliseconds), never with
another GPU result.  The 13B-class sample (tests/test_gpu_cfg5.py) does the
same at full size against stored oracle digests.
"""
import functools

import pytest

import workloads
from oracle.zkmat import prove_workload_group
from gpu_util import device_group

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_21393_amd import binding, serve
    binding.lib()
    return binding, serve


def _host_requests(n=8):
    """(list of workloads.Group, seed) per request; every request has two groups."""
    reqs = []
    for i in range(n):
        dims = [[(64, 128, 32)], [(70, 33, 130)], [(17, 64, 9), (17, 3, 9)], [(300, 520, 129)],
                [(5, 1, 3)], [(128, 1000, 64)]][i % 6]
        g = workloads.tiny_random_group(100 + i, dims, trans=(i % 2 == 1, i % 3 == 0), name=f"r{i}")
        g2 = workloads.tiny_random_group(200 + i, [(33, 40, 20)], name=f"s{i}")
        g.group_id, g2.group_id = 0, 1
        reqs.append(([g, g2], 1000 + i))
    return reqs


@functools.lru_cache(maxsize=None)
def _oracle_bytes(i):
    """The oracle's proofs of request i (request i does not depend on n)."""
    groups, seed = _host_requests(i + 1)[i]
    return [prove_workload_group(g, seed)[0] for g in groups]


def _requests(B, n=8):
    return [([device_group(g, B) for g in gs], seed) for gs, seed in _host_requests(n)]


def test_results_identical_alone_and_in_the_mix(env):
    B, serve = env
    reqs = _requests(B)
    for i, (gs, seed) in enumerate(reqs):
        assert B.sumcheck_matmul_prove(gs, seed, mode=B.VL_MODE_BATCHED)[0] == _oracle_bytes(i)
    srv = serve.ProofServer(n_slots=3, hbm_budget_bytes=1 << 30)
    for i, (gs, seed) in enumerate(reqs):
        srv.submit(serve.Request(i, gs, seed))
    srv.drain()
    assert srv.peak_in_flight >= 2
    for i in range(len(reqs)):
        r = srv.done[i]
        assert r.status == [0, 0]
        assert r.proofs == _oracle_bytes(i)


def test_budget_limits_admission(env):
    B, serve = env
    # four requests of one shape (other seeds): a budget of one request's bytes
    # admits exactly one at a time
    host = []
    for i in range(4):
        g = workloads.tiny_random_group(300 + i, [(64, 128, 32)], name=f"b{i}")
        host.append(([g], 2000 + i))
    reqs = [([device_group(g, B) for g in gs], seed) for gs, seed in host]
    sizer = serve.ProofServer(n_slots=1)
    need = sizer.request_bytes(serve.Request(0, *reqs[0]))
    assert all(sizer.request_bytes(serve.Request(0, *r)) == need for r in reqs)
    srv = serve.ProofServer(n_slots=4, hbm_budget_bytes=need)
    for i, (gs, seed) in enumerate(reqs):
        srv.submit(serve.Request(i, gs, seed))
    srv.drain()
    assert srv.peak_in_flight == 1
    for i, (gs, seed) in enumerate(host):
        assert srv.done[i].proofs == [prove_workload_group(g, seed)[0] for g in gs]


def test_false_statement_reported_per_request(env):
    B, serve = env
    g = workloads.tiny_random_group(7, [(8, 8, 8)])
    g.C = g.C.copy()
    g.C[0, 0] += 1
    good = workloads.tiny_random_group(8, [(8, 8, 8)])
    good.group_id = 1
    srv = serve.ProofServer(n_slots=2)
    srv.submit(serve.Request(0, [device_group(g, B), device_group(good, B)], 5))
    srv.drain()
    assert srv.done[0].status == [B.VL_ERR_FALSE_STATEMENT, 0]
    assert srv.done[0].proofs[1] == prove_workload_group(good, 5)[0]


def test_open_loop_poisson_arrivals(env):
    B, serve = env
    import numpy as np
    reqs = _requests(B, 6)
    gaps = np.random.default_rng(17).exponential(0.002, size=len(reqs))
    arrivals = [(float(t), i) for i, t in enumerate(np.cumsum(gaps))]
    srv = serve.ProofServer(n_slots=2)
    results, wall = serve.run_open_loop(srv, arrivals, lambda i, k: serve.Request(i, *reqs[k]))
    assert len(results) == len(reqs)
    summ = serve.latency_summary(results)
    assert summ["n"] == len(reqs) and summ["p99_ms"] >= summ["p50_ms"] > 0
    for r in results:
        assert r.proofs == _oracle_bytes(r.rid)


def test_one_slot_reuses_and_grows_its_buffers(env):
    B, serve = env
    # one slot, requests of different sizes in turn: the slot's pinned buffers
    # grow for the larger ones and are reused (and overwritten) by the others;
    # each result must still be that request's oracle proof
    reqs = _requests(B, 6)
    order = [4, 3, 0, 5, 4, 1, 3]          # small, large, mid, large, small, ...
    srv = serve.ProofServer(n_slots=1, hbm_budget_bytes=1 << 30)
    for i, k in enumerate(order):
        srv.submit(serve.Request(i, *reqs[k]))
    srv.drain()
    assert srv.peak_in_flight == 1
    sizes = set()
    for i, k in enumerate(order):
        expect = _oracle_bytes(k)
        assert srv.done[i].status == [0, 0]
        assert srv.done[i].proofs == expect
        sizes.add(sum(len(p) for p in expect))
    assert len(sizes) >= 3
    assert srv.slots[0].host_proofs.numel() == max(sizes)


def test_server_refuses_persistent_mode(env):
    B, serve = env
    reqs = _requests(B, 1)
    srv = serve.ProofServer(n_slots=1)
    with pytest.raises(ValueError):
        srv.submit(serve.Request(0, *reqs[0], mode=B.VL_MODE_PERSISTENT))


def test_planner_choice_is_used_and_bytes_unchanged(env):
    # the planner times launch shapes for a request's shape signature once;
    # the server then proves that shape with the cached choice, and the
    # proof bytes are the oracle's whatever the choice
    B, serve = env
    from paper_2508_21393_amd import tune
    g = workloads.tiny_random_group(41, [(70, 1030, 129)], name="plan")
    gs = [device_group(g, B)]
    planner = tune.Planner(grid=[(4096, 1, 2, 1), (16384, 2, 1, 0)], reps=1)
    rec = planner.plan(gs, 5)
    assert {"lane_macs", "segments", "cols_rows", "claim_order", "ms", "default_ms", "grid"} <= set(rec)
    assert planner.lookup(gs) is not None
    srv = serve.ProofServer(n_slots=2, planner=planner)
    for i in range(3):
        srv.submit(serve.Request(i, gs, 50 + i))
    srv.drain()
    for i in range(3):
        assert srv.done[i].proofs == [prove_workload_group(g, 50 + i)[0]]
