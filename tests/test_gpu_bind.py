"""Proofs bound to commitments, on the device (needs a gfx950 GPU).

A group's bind digest (32 bytes, typically a hash of its Hyrax commitments)
enters its transcript before the challenges u and v (Sec. II-C after
II-A).  Bound proofs must equal the oracle's bytes under the same digests in
every mode, through the asynchronous entry point and prove graphs (whose
digests can be replaced between launches), and the whole protocol must
close on the device: commit, prove bound to the commitments, verify the
sumcheck without a witness and check each reduced claim by an opening.
"""
import ctypes
import hashlib
import sys

import numpy as np
import pytest

import workloads
from oracle.zkmat import prove_workload_group
from gpu_util import to_dev

pytestmark = pytest.mark.gpu

CASES = [
    ([(8, 8, 8)], np.int16, (False, False), None),
    ([(6, 10, 5), (6, 3, 5)], np.int16, (True, False), None),
    ([(3, 8192, 5)], np.int16, (False, False), None),
    ([(5, 70, 9)], np.int32, (False, True), 14),
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


def _digest(tag, k):
    return hashlib.sha256(f"{tag}:{k}".encode()).digest()


def _groups():
    out = []
    for k, (dims, dt, trans, vb) in enumerate(CASES):
        g = workloads.tiny_random_group(300 + k, dims, dtype=dt, trans=trans, value_bits=vb, name=f"bind{k}")
        g.group_id = k
        out.append(g)
    return out


def _dev(B, g, bind):
    prods = [(to_dev(p.A), to_dev(p.B), p.transA, p.transB) for p in g.products]
    return B.GroupArgs(g.group_id, prods, to_dev(g.C), bind=bind)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_bound_proofs_match_oracle_bytes(B, mode):
    groups = _groups()
    binds = [_digest("m", k) if k != 1 else None for k in range(len(groups))]   # one group unbound
    _say(f"bound proofs mode={mode}")
    proofs, digests = B.sumcheck_matmul_prove([_dev(B, g, d) for g, d in zip(groups, binds)], 17, mode=mode)
    for g, d, pr, dg in zip(groups, binds, proofs, digests):
        op, st, _ = prove_workload_group(g, 17, bind=d)
        assert pr == op, g.name
        assert dg == st, g.name


def test_bound_async_and_graph_rebind(B):
    import torch
    groups = _groups()
    first = [_digest("a", k) for k in range(len(groups))]
    gs = [_dev(B, g, d) for g, d in zip(groups, first)]
    total = sum(B.proof_size(g) for g in gs)
    proofs = torch.zeros(total, dtype=torch.uint8, device="cuda")
    status = torch.full((len(gs),), -1, dtype=torch.int32, device="cuda")
    ws = torch.empty(B.workspace_size(gs, 1, async_=True), dtype=torch.uint8, device="cuda")
    _say("bound async")
    offs = B.sumcheck_matmul_prove_async(gs, 4, proofs, status, ws, mode=1)
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [0] * len(gs)
    raw = proofs.cpu().numpy().tobytes()
    for i, (g, d) in enumerate(zip(groups, first)):
        assert raw[offs[i]:offs[i + 1]] == prove_workload_group(g, 4, bind=d)[0], g.name

    second = [_digest("b", k) for k in range(len(groups))]
    _say("bound prove graph")
    with B.ProveGraph(gs, ws, proofs, status) as G:
        # the graph copied the digests at create: overwriting the caller's
        # buffers afterwards changes nothing
        for ga in gs:
            ctypes.memmove(ga._bind, b"\xff" * 32, 32)
        for binds, seed in ((first, 4), (second, 5), (None, 5), (second, 6)):
            if binds is not first:
                G.bind(binds)
            proofs.zero_()
            status.fill_(-1)
            G.launch(seed)
            torch.cuda.synchronize()
            assert status.cpu().tolist() == [0] * len(groups)
            raw = proofs.cpu().numpy().tobytes()
            for i, g in enumerate(groups):
                d = None if binds is None else binds[i]
                assert raw[G.offsets[i]:G.offsets[i + 1]] == prove_workload_group(g, seed, bind=d)[0], (seed, i)


def test_commit_prove_open_on_the_device(B):
    # Hyrax row commitments of A, B and C on the device, a proof bound to
    # their digest, the host verifier without a witness, and each reduced
    # claim checked by a device opening against its commitment
    import torch
    rng = np.random.default_rng(41)
    D0, D1, D2 = 8, 4096, 4
    A = rng.integers(-2 ** 15, 2 ** 15, size=(D0, D1)).astype(np.int16)
    Bm = rng.integers(-2 ** 15, 2 ** 15, size=(D1, D2)).astype(np.int16)
    C = A.astype(np.int64) @ Bm.astype(np.int64)
    Ad, Bd, Cd = to_dev(A), to_dev(Bm), to_dev(C)
    _say("commit, prove, open")
    table = B.HyraxTable(D1, windows=8)
    cA, cB, cC = (B.hyrax_commit(M, table) for M in (Ad, Bd, Cd))
    torch.cuda.synchronize()
    enc = [c.cpu().numpy().tobytes() for c in (cA, cB, cC)]
    d = hashlib.sha256(b"".join(enc)).digest()
    g = workloads.Group("committed", [workloads.Product("AB", A, Bm)], C, 0)
    proofs, _ = B.sumcheck_matmul_prove([B.GroupArgs(0, [(Ad, Bd, False, False)], Cd, bind=d)], 8, mode=1)
    assert proofs[0] == prove_workload_group(g, 8, bind=d)[0]

    ok, fr, red = B.verify_transcript(proofs[0], B.GroupArgs.shapes_only(0, [(D0, D1, D2)], bind=d), 8)
    assert ok, B.last_error()
    n0, n1, n2 = 3, 12, 2
    c, u, v = red[0], red[1:1 + n0], red[1 + n0:1 + n0 + n2]
    r = red[1 + n0 + n2:1 + n0 + n2 + n1]
    af, bf = red[1 + n0 + n2 + n1], red[2 + n0 + n2 + n1]

    def opened(commits, M, x, y):
        R, m = M.shape
        okk, val, msg = B.hyrax_verify_open(commits, R, m, x, y, B.hyrax_open(M, x))
        assert okk, msg
        return val

    assert opened(enc[0], Ad, u, r) == af
    assert opened(enc[1], Bd, r, v) == bf
    assert opened(enc[2], Cd, u, v) == c
