"""Host side of the Hyrax commitments (no GPU): the library's generators
against the oracle's, its opening verifier against oracle commitments and
openings (accepts, returns the MLE value, rejects every tamper), and the
argument checks of the device entry points (they fail before touching the
device)."""
import os
import random

import numpy as np
import pytest

import oracle.hyrax as hy
from oracle import P, matrix_mle
from oracle.mle import num_vars
from paper_2508_21393_amd import binding as B


def _lib_or_skip():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libverilora.so not built")
    return B.lib()


def test_generators_match_the_oracle():
    _lib_or_skip()
    m = 24
    g = B.hyrax_generators(m)
    for j in range(m):
        assert hy.decode(g[96 * j:96 * j + 96]) == hy.generator(j), j


def _case(seed, R, m, lo=-(1 << 15), hi=1 << 15):
    rng = np.random.default_rng(seed)
    M = rng.integers(lo, hi, size=(R, m)).astype(np.int64)
    gens = hy.generators(m)
    C = hy.commit(M, gens)
    r = random.Random(seed)
    x = [r.randrange(P) for _ in range(num_vars(R))]
    y = [r.randrange(P) for _ in range(num_vars(m))]
    return M, gens, C, x, y


def _enc(C):
    return b"".join(hy.encode(c) for c in C)


@pytest.mark.parametrize("R,m", [(4, 8), (3, 5), (1, 1), (1, 6), (7, 1), (5, 9)])
def test_verifier_accepts_oracle_openings(R, m):
    _lib_or_skip()
    M, gens, C, x, y = _case(R * 31 + m, R, m)
    w = hy.open_at(M, x)
    ok, val, msg = B.hyrax_verify_open(_enc(C), R, m, x, y, w)
    assert ok, msg
    assert val == matrix_mle(M, x, y) == hy.verify_open(C, gens, x, y, w)


def test_verifier_accepts_zero_rows():
    _lib_or_skip()
    M, gens, C, x, y = _case(3, 4, 6)
    M[1] = 0
    C = hy.commit(M, gens)
    assert C[1] is None
    w = hy.open_at(M, x)
    ok, val, msg = B.hyrax_verify_open(_enc(C), 4, 6, x, y, w)
    assert ok, msg
    assert val == matrix_mle(M, x, y)


def test_verifier_rejects_tampering():
    _lib_or_skip()
    R, m = 4, 6
    M, gens, C, x, y = _case(11, R, m)
    w = hy.open_at(M, x)
    enc = _enc(C)
    # a changed opening element
    for j in (0, m - 1):
        bad = list(w)
        bad[j] = (bad[j] + 1) % P
        ok, _, msg = B.hyrax_verify_open(enc, R, m, x, y, bad)
        assert not ok and "does not match" in msg
    # a commitment moved by a generator (still a valid point)
    Cb = list(C)
    Cb[2] = hy.add(Cb[2], gens[0])
    ok, _, msg = B.hyrax_verify_open(_enc(Cb), R, m, x, y, w)
    assert not ok and "does not match" in msg
    # the opening for another point
    ok, _, _ = B.hyrax_verify_open(enc, R, m, [(v + 1) % P for v in x], y, w)
    assert not ok
    # a byte flipped: off the curve
    raw = bytearray(enc)
    raw[96 + 7] ^= 1
    ok, _, msg = B.hyrax_verify_open(bytes(raw), R, m, x, y, w)
    assert not ok and "curve point" in msg
    # a non-canonical coordinate (y + q < 2^384 names the same field element)
    X, Y = C[0]
    raw = bytearray(enc)
    raw[48:96] = (Y + hy.Q).to_bytes(48, "little")
    ok, _, msg = B.hyrax_verify_open(bytes(raw), R, m, x, y, w)
    assert not ok and "curve point" in msg
    # a non-canonical field element in the opening
    bad = list(w)
    bad[0] += P
    ok, _, msg = B.hyrax_verify_open(enc, R, m, x, y, bad)
    assert not ok and "canonical" in msg


def test_verifier_rejects_points_outside_the_subgroup():
    _lib_or_skip()
    # a curve point that is not in the order-p subgroup (no cofactor clearing)
    X = 7
    while True:
        s = (X ** 3 + hy.B_COEF) % hy.Q
        if pow(s, (hy.Q - 1) // 2, hy.Q) == 1:
            break
        X += 1
    Pt = (X, pow(s, (hy.Q + 1) // 4, hy.Q))
    assert hy.on_curve(Pt) and hy.mul(P, Pt) is not None
    R, m = 2, 3
    M, gens, C, x, y = _case(5, R, m)
    w = hy.open_at(M, x)
    ok, _, msg = B.hyrax_verify_open(hy.encode(Pt) + hy.encode(C[1]), R, m, x, y, w)
    assert not ok and "outside the group" in msg


def test_size_queries_and_argument_checks():
    L = _lib_or_skip()
    assert B.hyrax_table_size(10, 2) == 10 * 2 * 128 * 96
    assert B.hyrax_table_size(0, 2) == 0 and B.hyrax_table_size(10, 0) == 0 and B.hyrax_table_size(10, 9) == 0
    assert B.hyrax_table_size((1 << 20) + 1, 2) == 0
    assert B.hyrax_commit_workspace_size(4096, 4096) > 0
    assert B.hyrax_commit_workspace_size(0, 16) == 0
    # the commit call checks its arguments before any device work (the
    # pointers below are never dereferenced)
    fake = 1 << 20
    assert L.vl_hyrax_commit(fake, 7, 4, 8, 8, fake, 8, 2, 0, fake, fake, 1 << 20, None) == B.VL_ERR_DTYPE
    assert L.vl_hyrax_commit(fake, 1, 4, 9, 9, fake, 8, 2, 0, fake, fake, 1 << 20, None) == B.VL_ERR_SHAPE
    assert L.vl_hyrax_commit(fake, 2, 4, 8, 8, fake, 8, 2, 0, fake, fake, 1 << 20, None) == B.VL_ERR_INVALID_ARG
    assert L.vl_hyrax_commit(fake, 1, 4, 8, 7, fake, 8, 2, 0, fake, fake, 1 << 20, None) == B.VL_ERR_SHAPE
    assert L.vl_hyrax_commit(fake, 1, 4, 8, 8, fake, 8, 2, 0, fake, fake, 16, None) == B.VL_ERR_WORKSPACE
    assert L.vl_hyrax_commit(fake, 1, 4, 8, 8, fake, 8, 2, 2, fake, fake, 1 << 20, None) == B.VL_ERR_INVALID_ARG
    assert L.vl_hyrax_commit(None, 1, 4, 8, 8, fake, 8, 2, 0, fake, fake, 1 << 20, None) == B.VL_ERR_INVALID_ARG
    assert L.vl_hyrax_setup(0, 2, fake, 1 << 30, None) == B.VL_ERR_SHAPE
    assert L.vl_hyrax_setup(4, 2, fake, 16, None) == B.VL_ERR_BUFFER_TOO_SMALL
