"""Continuous-batching server: each result is the same alone and in the mix."""
import numpy as np
import pytest

import workloads
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


def _requests(B, n=8):
    reqs = []
    for i in range(n):
        dims = [[(64, 128, 32)], [(70, 33, 130)], [(17, 64, 9), (17, 3, 9)], [(300, 520, 129)],
                [(5, 1, 3)], [(128, 1000, 64)]][i % 6]
        g = workloads.tiny_random_group(100 + i, dims, trans=(i % 2 == 1, i % 3 == 0), name=f"r{i}")
        g2 = workloads.tiny_random_group(200 + i, [(33, 40, 20)], name=f"s{i}")
        g.group_id, g2.group_id = 0, 1
        reqs.append(([device_group(g, B), device_group(g2, B)], 1000 + i))
    return reqs


def test_results_identical_alone_and_in_the_mix(env):
    B, serve = env
    reqs = _requests(B)
    alone = [B.sumcheck_matmul_prove(gs, seed, mode=B.VL_MODE_BATCHED)[0] for gs, seed in reqs]
    srv = serve.ProofServer(n_slots=3, hbm_budget_bytes=1 << 30)
    for i, (gs, seed) in enumerate(reqs):
        srv.submit(serve.Request(i, gs, seed))
    srv.drain()
    assert srv.peak_in_flight >= 2
    for i in range(len(reqs)):
        r = srv.done[i]
        assert r.status == [0, 0]
        assert r.proofs == alone[i]


def test_budget_limits_admission(env):
    B, serve = env
    # four requests of one shape (other seeds): a budget of one request's bytes
    # admits exactly one at a time
    reqs = []
    for i in range(4):
        g = workloads.tiny_random_group(300 + i, [(64, 128, 32)], name=f"b{i}")
        reqs.append(([device_group(g, B)], 2000 + i))
    need = serve.ProofServer.request_bytes(serve.Request(0, *reqs[0]))
    assert all(serve.ProofServer.request_bytes(serve.Request(0, *r)) == need for r in reqs)
    srv = serve.ProofServer(n_slots=4, hbm_budget_bytes=need)
    for i, (gs, seed) in enumerate(reqs):
        srv.submit(serve.Request(i, gs, seed))
    srv.drain()
    assert srv.peak_in_flight == 1
    for i, (gs, seed) in enumerate(reqs):
        assert srv.done[i].proofs == B.sumcheck_matmul_prove(gs, seed, mode=B.VL_MODE_BATCHED)[0]


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


def test_open_loop_poisson_arrivals(env):
    B, serve = env
    reqs = _requests(B, 6)
    arrivals = [(0.002 * i, i) for i in range(len(reqs))]
    srv = serve.ProofServer(n_slots=2)
    results, wall = serve.run_open_loop(srv, arrivals, lambda i, k: serve.Request(i, *reqs[k]))
    assert len(results) == len(reqs)
    summ = serve.latency_summary(results)
    assert summ["n"] == len(reqs) and summ["p99_ms"] >= summ["p50_ms"] > 0
    for r in results:
        assert r.proofs == B.sumcheck_matmul_prove(*reqs[r.rid], mode=B.VL_MODE_BATCHED)[0]


def test_one_slot_reuses_and_grows_its_buffers(env):
    B, serve = env
    # one slot, requests of different sizes in turn: the slot's pinned buffers
    # grow for the larger ones and are reused (and overwritten) by the others;
    # each result must still be that request's own solo proof
    reqs = _requests(B, 6)
    order = [4, 3, 0, 5, 4, 1, 3]          # small, large, mid, large, small, ...
    srv = serve.ProofServer(n_slots=1, hbm_budget_bytes=1 << 30)
    for i, k in enumerate(order):
        srv.submit(serve.Request(i, *reqs[k]))
    srv.drain()
    assert srv.peak_in_flight == 1
    sizes = set()
    for i, k in enumerate(order):
        gs, seed = reqs[k]
        expect = B.sumcheck_matmul_prove(gs, seed, mode=B.VL_MODE_BATCHED)[0]
        assert srv.done[i].status == [0, 0]
        assert srv.done[i].proofs == expect
        sizes.add(sum(len(p) for p in expect))
    assert len(sizes) >= 3
    assert srv.slots[0].host_proofs.numel() == max(sizes)
