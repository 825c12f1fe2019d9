"""13B-class serving sample against the oracle (needs a gfx950 GPU).

The fixed request mix of workloads.serving_sample (every target, T in
{128, 512, 2048}, rank in {8, 16, 64}, forward / backward / update types;
hidden 5120 padded to 8192, FFN 13824 padded to 16384) is proved alone and
then through the continuous-batching server with Poisson arrivals.  Every
group's proof bytes (SHA-256) and final transcript state must equal what the
CPU oracle computed for the same request (tests/golden/cfg5.json, written by
tests/golden/make_golden.py, which runs only the oracle).
"""
import sys

import numpy as np
import pytest

import workloads
from gpu_util import device_group, golden, sha

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sample():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_21393_amd import binding as B, serve
    B.lib()
    gold = golden("cfg5")
    specs = workloads.serving_sample(gold["n"])
    weights, reqs = {}, []
    for k, sp in enumerate(specs):
        rec = gold["requests"][k]
        assert (rec["target"], rec["T"], rec["rank"], rec["kind"]) == sp
        _say(f"cfg5: generating request {k} {sp}")
        # witness products as exact float64 GEMMs on the GPU
        w = workloads.serving_sample_workload(k, sp, weights, device="cuda")
        assert w.seed == rec["seed"]
        reqs.append((w, [device_group(g, B) for g in w.groups], rec))
    return B, serve, reqs


def _check(groups_bytes, digests, rec, k):
    assert len(groups_bytes) == len(rec["groups"])
    for i, (pr, g) in enumerate(zip(groups_bytes, rec["groups"])):
        assert sha(pr) == g["proof_sha256"], (k, g["name"])
        if digests is not None:
            assert digests[i].hex() == g["state"], (k, g["name"])


def test_cfg5_requests_alone_match_oracle(sample):
    B, _, reqs = sample
    for k, (w, gs, rec) in enumerate(reqs):
        _say(f"cfg5: request {k} alone ({rec['kind']} {rec['target']} T={rec['T']} r={rec['rank']})")
        proofs, digests = B.sumcheck_matmul_prove(gs, w.seed, mode=B.VL_MODE_BATCHED)
        _check(proofs, digests, rec, k)


def test_cfg5_requests_served_match_oracle(sample):
    # three slots, Poisson arrivals faster than one request's service time, so
    # requests overlap on the device; every request twice, in a shuffled order
    B, serve, reqs = sample
    rng = np.random.default_rng(55)
    order = list(range(len(reqs))) * 2
    rng.shuffle(order)
    gaps = rng.exponential(0.0005, size=len(order))
    arrivals = [(float(t), k) for t, k in zip(np.cumsum(gaps), order)]
    srv = serve.ProofServer(n_slots=3, hbm_budget_bytes=32 << 30)
    _say(f"cfg5: serving {len(arrivals)} arrivals")
    results, _ = serve.run_open_loop(srv, arrivals,
                                     lambda i, k: serve.Request(i, reqs[k][1], reqs[k][0].seed))
    assert srv.peak_in_flight >= 2
    assert len(results) == len(arrivals)
    for r in results:
        k = arrivals[r.rid][1]
        assert r.status == [0] * len(reqs[k][1]), k
        _check(r.proofs, None, reqs[k][2], k)
