"""Parity of the wide matmul rounds with the CPU oracle (needs a gfx950 GPU).

A group whose first product has an inner dimension of 8192 or more (padded:
its round 2 then has 2048 pairs or more) proves its first rounds across the
whole GPU: one sweep launch per round,
whose blocks each take the previous round's transcript step, fold the
tables and sum the next round's pairs.  The proof bytes must not change:
every case here compares them, exactly, with the oracle's proof of the same
seeded group (Sec. III-B, the matmul sumcheck; tolerance 0), including the
refusals the first round decides (a false claim, an out-of-range claim
entry), batches that mix wide and narrow groups, repeated calls on one
workspace, and graph replays.
"""
import sys

import numpy as np
import pytest

import workloads
from oracle.zkmat import prove_workload_group
from gpu_util import device_group

pytestmark = pytest.mark.gpu

# (dims of the products, dtype, transposed views, value bits): first
# products with D1 = 8192 .. 16384 (three or four wide rounds), ragged D1,
# a second narrow product in the group, and every entry type (value bits
# keep every claim entry within |x| < 2^47)
WIDE_CASES = [
    ([(3, 8192, 5)], np.int16, (False, False), None),
    ([(4, 8192, 3), (4, 16, 3)], np.int16, (False, False), None),
    ([(5, 5000, 7)], np.int32, (True, False), 14),
    ([(2, 16384, 2)], np.int16, (False, True), None),
    ([(6, 4100, 4), (6, 4100, 4)], np.int64, (True, True), 16),
]


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


def _groups(cases=WIDE_CASES, seed0=100):
    out = []
    for k, (dims, dt, trans, vb) in enumerate(cases):
        g = workloads.tiny_random_group(seed0 + k, dims, dtype=dt, trans=trans, value_bits=vb, name=f"wide{k}")
        g.group_id = k
        out.append(g)
    return out


def _oracle(groups, seed):
    return [prove_workload_group(g, seed)[:2] for g in groups]


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_wide_groups_match_oracle_bytes(B, mode):
    # per-instance, batched and persistent (which keeps the rounds in its
    # resident launch) must all give the oracle's bytes
    groups = _groups()
    _say(f"wide groups mode={mode}")
    proofs, digests = B.sumcheck_matmul_prove([device_group(g, B) for g in groups], 21, mode=mode)
    for g, pr, dg, (op, st) in zip(groups, proofs, digests, _oracle(groups, 21)):
        assert pr == op, g.name
        assert dg == st, g.name


@pytest.mark.parametrize("segments", [2, 3])
def test_wide_groups_across_segments(B, segments):
    # groups cut into pipeline segments: each segment launches its own
    # groups' wide rounds
    groups = _groups()
    _say(f"wide groups segments={segments}")
    proofs, _ = B.sumcheck_matmul_prove([device_group(g, B) for g in groups], 5, mode=1,
                                        tuning_=B.tuning(segments=segments))
    for g, pr, (op, _) in zip(groups, proofs, _oracle(groups, 5)):
        assert pr == op, g.name


@pytest.mark.parametrize("dtype,delta", [(np.int16, -1), (np.int64, 1 << 60)])
def test_wide_false_statement_refused(B, dtype, delta):
    g = workloads.tiny_random_group(31, [(3, 8192, 5)], dtype=dtype, value_bits=None if dtype == np.int16 else 12)
    g.C = g.C.copy()
    g.C[2, 4] += delta
    _say(f"wide false statement {np.dtype(dtype).name}")
    with pytest.raises(B.VLError) as e:
        B.sumcheck_matmul_prove([device_group(g, B)], 1, mode=1)
    assert e.value.status == B.VL_ERR_FALSE_STATEMENT


def test_wide_range_error_on_oversized_claim_entry(B):
    # int16 factors: C is contracted in two 24-bit digits, so an entry
    # beyond |x| < 2^47 is refused (int64 factors take three digits, which
    # cover every int64 entry: there the same C is a false statement)
    g = workloads.tiny_random_group(32, [(4, 8192, 3)])
    g.C = g.C.copy()
    g.C[3, 0] = 1 << 60
    _say("wide range error")
    with pytest.raises(B.VLError) as e:
        B.sumcheck_matmul_prove([device_group(g, B)], 1, mode=1)
    assert e.value.status == B.VL_ERR_RANGE


def test_wide_async_mixed_batch_statuses(B):
    # a batch of valid and refused groups, wide and narrow: each group's
    # status word is its own, and the valid groups' bytes are the oracle's
    import torch
    cases = [
        ([(3, 8192, 5)], np.int16, (False, False), None),     # valid, wide
        ([(2, 8192, 2)], np.int16, (False, False), None),     # false claim, wide
        ([(8, 8, 8)], np.int16, (False, False), None),        # valid, narrow
        ([(4, 8192, 3)], np.int16, (False, False), None),     # range error, wide
        ([(5, 5000, 7)], np.int32, (True, False), 14),        # valid, wide
    ]
    groups = _groups(cases, seed0=200)
    groups[1].C = groups[1].C.copy()
    groups[1].C[0, 1] += 3
    groups[3].C = groups[3].C.copy()
    groups[3].C[1, 2] = -(1 << 60)
    gs = [device_group(g, B) for g in groups]
    total = sum(B.proof_size(g) for g in gs)
    proofs = torch.zeros(total, dtype=torch.uint8, device="cuda")
    status = torch.full((len(gs),), -1, dtype=torch.int32, device="cuda")
    ws = torch.empty(B.workspace_size(gs, 1, async_=True), dtype=torch.uint8, device="cuda")
    _say("wide async mixed batch")
    offs = B.sumcheck_matmul_prove_async(gs, 9, proofs, status, ws, mode=1)
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [0, B.VL_ERR_FALSE_STATEMENT, 0, B.VL_ERR_RANGE, 0]
    raw = proofs.cpu().numpy().tobytes()
    for i in (0, 2, 4):
        assert raw[offs[i]:offs[i + 1]] == prove_workload_group(groups[i], 9)[0], groups[i].name


def test_wide_repeated_calls_reuse_workspace(B):
    # the rounds' counters and transcript slots live in the call's
    # descriptors and start from zero on every call: calls on one
    # workspace, with new seeds and new data, each give the oracle's bytes
    import torch
    groups = _groups()
    gs = [device_group(g, B) for g in groups]
    total = sum(B.proof_size(g) for g in gs)
    proofs = torch.zeros(total, dtype=torch.uint8, device="cuda")
    status = torch.full((len(gs),), -1, dtype=torch.int32, device="cuda")
    ws = torch.empty(B.workspace_size(gs, 1, async_=True), dtype=torch.uint8, device="cuda")
    for it, seed in enumerate((3, 4, 4, 11)):
        if it == 2:
            # new data in the same device tensors (a valid statement again)
            g = workloads.tiny_random_group(77, [(3, 8192, 5)], name="wide0")
            g.group_id = 0
            C_d, A_d, B_d = gs[0].keep
            A_d.copy_(torch.from_numpy(g.products[0].A))
            B_d.copy_(torch.from_numpy(g.products[0].B))
            C_d.copy_(torch.from_numpy(g.C))
            groups[0] = g
        _say(f"wide repeated call seed={seed}")
        proofs.zero_()
        status.fill_(-1)
        offs = B.sumcheck_matmul_prove_async(gs, seed, proofs, status, ws, mode=1)
        torch.cuda.synchronize()
        assert status.cpu().tolist() == [0] * len(gs)
        raw = proofs.cpu().numpy().tobytes()
        for i, (op, _) in enumerate(_oracle(groups, seed)):
            assert raw[offs[i]:offs[i + 1]] == op, (seed, groups[i].name)


@pytest.mark.parametrize("segments", [1, 3])
def test_wide_prove_graph_replays_match_oracle(B, segments):
    import torch
    groups = _groups()
    gs = [device_group(g, B) for g in groups]
    total = sum(B.proof_size(g) for g in gs)
    proofs = torch.zeros(total, dtype=torch.uint8, device="cuda")
    status = torch.full((len(gs),), -1, dtype=torch.int32, device="cuda")
    digests = torch.zeros(32 * len(gs), dtype=torch.uint8, device="cuda")
    tn = B.tuning(segments=segments)
    ws = torch.empty(B.workspace_size(gs, 1, async_=True, tuning_=tn), dtype=torch.uint8, device="cuda")
    _say(f"wide prove graph segments={segments}")
    with B.ProveGraph(gs, ws, proofs, status, digests_dev=digests, tuning_=tn) as G:
        for seed in (13, 14, 13):
            proofs.zero_()
            status.fill_(-1)
            G.launch(seed)
            torch.cuda.synchronize()
            assert status.cpu().tolist() == [0] * len(gs)
            raw = proofs.cpu().numpy().tobytes()
            dg = digests.cpu().numpy().tobytes()
            # eager work between replays
            B.sumcheck_matmul_prove(gs[:1], seed + 1, mode=1)
            for i, (op, st) in enumerate(_oracle(groups, seed)):
                assert raw[G.offsets[i]:G.offsets[i + 1]] == op, (seed, i)
                assert dg[32 * i:32 * i + 32] == st, (seed, i)
