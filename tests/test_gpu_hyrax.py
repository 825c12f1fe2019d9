"""Hyrax commitments on the GPU against the oracle (needs a gfx950 GPU).

vl_hyrax_setup must write the oracle's generators and every table point
k 256^w G_j; vl_hyrax_commit must write the oracle's commitment bytes
(oracle/hyrax.py) for int16, int32 and int64 matrices of ragged shapes,
with every column split, zero rows and the extreme values of each type;
at the 7B-class size (4096 x 4096 int16 weights) sampled rows are checked
against the oracle, all rows through additivity, and an opening computed
on the device (partial evaluation) passes the host verifier with the
oracle's MLE value.
"""
import random
import sys

import numpy as np
import pytest

import oracle.hyrax as hy
import workloads
from oracle import P
from oracle.mle import eq_table, num_vars

pytestmark = pytest.mark.gpu

RINV = pow(1 << 384, -1, hy.Q)


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


_GENS = {}


def gens(m):
    """oracle generators, computed once per process"""
    have = _GENS.setdefault("g", [])
    while len(have) < m:
        have.append(hy.generator(len(have)))
    return have[:m]


def _table_point(buf, W, j, w, k):
    """(x, y) of table point k 256^w G_j from the device table (Montgomery)"""
    off = (((j * W + w) * 128) + k - 1) * 96
    x = int.from_bytes(buf[off:off + 48], "little") * RINV % hy.Q
    y = int.from_bytes(buf[off + 48:off + 96], "little") * RINV % hy.Q
    return (x, y)


@pytest.mark.parametrize("m,W", [(5, 2), (3, 8)])
def test_setup_table_matches_oracle(B, m, W):
    import torch
    _say(f"hyrax setup m={m} W={W}")
    T = B.HyraxTable(m, W)
    torch.cuda.synchronize()
    buf = T.buf.cpu().numpy().tobytes()
    G = gens(m)
    rng = random.Random(m * 10 + W)
    for j in range(m):
        assert _table_point(buf, W, j, 0, 1) == G[j], j
        ks = range(1, 129) if W == 2 else rng.sample(range(1, 129), 6) + [1, 128]
        for w in range(W):
            for k in ks:
                assert _table_point(buf, W, j, w, k) == hy.mul(k << (8 * w), G[j]), (j, w, k)


def _commit_dev(B, T, M, split=0):
    import torch
    Md = torch.from_numpy(np.ascontiguousarray(M)).cuda()
    out = B.hyrax_commit(Md, T, split=split)
    torch.cuda.synchronize()
    return out.cpu().numpy().tobytes()


def _expect(M, m):
    return b"".join(hy.encode(c) for c in hy.commit(M.astype(np.int64), gens(m)))


_TABLES = {}


def table(B, m, W):
    key = (m, W)
    if key not in _TABLES:
        _TABLES[key] = B.HyraxTable(m, W)
    return _TABLES[key]


CASES = [  # (R, m, dtype, split)
    (3, 5, np.int16, 0), (9, 130, np.int16, 0), (9, 130, np.int16, 2), (9, 130, np.int16, 3),
    (1, 1, np.int16, 0), (2, 64, np.int16, 1), (4, 70, np.int32, 0), (2, 65, np.int64, 0), (5, 200, np.int16, 4),
]


@pytest.mark.parametrize("R,m,dt,split", CASES)
def test_commit_matches_oracle(B, R, m, dt, split):
    _say(f"hyrax commit R={R} m={m} {np.dtype(dt).name} split={split}")
    rng = np.random.default_rng(R * 1000 + m + split)
    info = np.iinfo(dt)
    lo, hi = (info.min, info.max) if dt == np.int16 else (-(1 << 20), 1 << 20)
    M = rng.integers(lo, hi, size=(R, m), endpoint=True).astype(dt)
    T = table(B, 256, 8)
    assert _commit_dev(B, T, M, split) == _expect(M, m)


@pytest.mark.parametrize("dt", [np.int16, np.int32, np.int64])
def test_commit_extreme_values_and_zero_rows(B, dt):
    _say(f"hyrax commit extremes {np.dtype(dt).name}")
    info = np.iinfo(dt)
    vals = [info.min, info.max, info.min + 1, info.max - 1, 0, 1, -1, 127, 128, -128, -129, 255, 256, -256]
    m = 70
    M = np.zeros((4, m), dtype=dt)
    M[0, :len(vals)] = vals
    M[2, :] = info.max
    M[3, :] = info.min
    M[3, 5] = 0
    T = table(B, 256, 8)
    got = _commit_dev(B, T, M)
    assert got[96:192] == bytes(96)          # a zero row commits to the point at infinity
    assert got == _expect(M, m)


def test_commit_cancelling_entries(B):
    # v G_j + (-v) G_j in one row: the lane sums meet equal and opposite
    # points, and a row of one generator's multiples doubles
    _say("hyrax commit cancellation")
    m = 130
    M = np.zeros((3, m), dtype=np.int16)
    M[0, 0], M[0, 64] = 5, -5            # different generators: no cancellation
    M[1, 3] = 1
    M[2, :] = 1
    T = table(B, 256, 8)
    assert _commit_dev(B, T, M) == _expect(M, m)


def test_table_with_more_generators_and_windows_than_needed(B):
    _say("hyrax commit with a larger table")
    rng = np.random.default_rng(9)
    M = rng.integers(-300, 300, size=(3, 40)).astype(np.int16)
    assert _commit_dev(B, table(B, 256, 8), M) == _commit_dev(B, table(B, 64, 2), M) == _expect(M, 40)


def test_full_size_weights_sampled_rows_additivity_and_opening(B):
    import torch
    _say("hyrax 7B-class W_q 4096 x 4096: commit")
    (_, W), = workloads.block_weights(only=["q"])
    R, m = W.shape
    T = table(B, m, 2)
    Wd = torch.from_numpy(W).cuda()
    C = B.hyrax_commit(Wd, T)
    torch.cuda.synchronize()
    Cb = C.cpu().numpy().tobytes()
    # two rows against the oracle, entry by entry
    G = gens(m)
    for i in (0, R - 1):
        _say(f"  oracle row {i}")
        assert Cb[96 * i:96 * i + 96] == hy.encode(hy.commit(W[i:i + 1].astype(np.int64), G)[0]), i
    # every row: commit(W + D) = commit(W) + commit(D) for a random D
    _say("  additivity")
    rng = np.random.default_rng(2)
    D = rng.integers(-2000, 2000, size=W.shape).astype(np.int16)
    C_D = B.hyrax_commit(torch.from_numpy(D).cuda(), T).cpu().numpy().tobytes()
    C_S = B.hyrax_commit(torch.from_numpy((W.astype(np.int32) + D).astype(np.int16)).cuda(), T).cpu().numpy().tobytes()
    for i in rng.choice(R, 64, replace=False):
        s = slice(96 * i, 96 * i + 96)
        assert hy.add(hy.decode(Cb[s]), hy.decode(C_D[s])) == hy.decode(C_S[s]), i
    # an opening at a random point from the device partial evaluation
    _say("  opening")
    r = random.Random(5)
    x = [r.randrange(P) for _ in range(num_vars(R))]
    y = [r.randrange(P) for _ in range(num_vars(m))]
    w = B.hyrax_open(Wd, x)
    w_oracle = hy.open_at(W, x)
    assert w == [int(v) % P for v in w_oracle]
    ok, val, msg = B.hyrax_verify_open(Cb, R, m, x, y, w)
    assert ok, msg
    assert val == sum(int(a) * b for a, b in zip(w_oracle, eq_table(y))) % P
    bad = list(w)
    bad[17] = (bad[17] + 1) % P
    assert not B.hyrax_verify_open(Cb, R, m, x, y, bad)[0]
