"""The allocation-free partial evaluation against the workspace one (needs a GPU).

vl_mle_partial_eval_noalloc takes its scratch from a fixed device array of
the library.  Two calls in a row (the second on a smaller input, so the
array still holds the first call's larger contents) must each give exactly
the words vl_mle_partial_eval gives on the same inputs, which the parity
tests tie to the oracle; one case is also checked against the oracle here.
Shapes whose scratch would not fit are refused before any device work.
"""
import ctypes
import random
import sys

import numpy as np
import pytest

import oracle
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


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


def _case(B, rows, cols, contract, dtype, bits, seed):
    import torch
    rng = np.random.default_rng(seed)
    M = rng.integers(-(1 << bits), 1 << bits, size=(rows, cols), dtype=np.int64).astype(dtype)
    len_ = rows if contract == 0 else cols
    nv = oracle.num_vars(len_)
    prng = random.Random(seed)
    pt = [prng.randrange(oracle.P) for _ in range(nv)]
    eq = torch.empty((8, 1 << nv), dtype=torch.int32, device="cuda")
    B.eq_table(pt, B.fr_vec(eq))
    L = 1 << oracle.num_vars(cols if contract == 0 else rows)
    return M, to_dev(M), pt, eq, L


def _both(B, rows, cols, contract, dtype, bits, seed):
    """(workspace result, no-alloc result, host matrix, point) as int32 tensors."""
    import torch
    M, Md, pt, eq, L = _case(B, rows, cols, contract, dtype, bits, seed)
    ref = torch.full((8, L), 7, dtype=torch.int32, device="cuda")
    ws = torch.empty(B.partial_eval_workspace_size(rows, cols, contract, M.dtype), dtype=torch.uint8, device="cuda")
    B.mle_partial_eval(Md, contract, B.fr_vec(eq), B.fr_vec(ref), ws)
    got = torch.full((8, L), 5, dtype=torch.int32, device="cuda")
    B.mle_partial_eval_noalloc(Md, contract, B.fr_vec(eq), B.fr_vec(got))
    torch.cuda.synchronize()
    return ref.cpu(), got.cpu(), M, pt


# (rows, cols, contract, dtype, bits): the first of each pair needs the larger
# scratch (split contractions with chunk partials), the second is smaller
PAIRS = [
    ((4096, 2048, 0, np.int16, 15), (300, 130, 1, np.int16, 15)),
    ((2048, 11008, 1, np.int16, 15), (70, 33, 0, np.int16, 15)),
    ((3000, 777, 0, np.int64, 44), (17, 260, 1, np.int64, 40)),
]


@pytest.mark.parametrize("big,small", PAIRS)
def test_noalloc_matches_workspace_entry_point_twice(B, big, small):
    for k, shape in enumerate((big, small)):
        _say(f"noalloc call {k}: rows={shape[0]} cols={shape[1]} contract={shape[2]} dtype={shape[3].__name__}")
        ref, got, _, _ = _both(B, *shape, seed=1000 * k + shape[0])
        assert bool((ref == got).all()), (k, shape)


def test_noalloc_matches_oracle(B):
    _say("noalloc vs oracle: rows=300 cols=130 contract=0")
    ref, got, M, pt = _both(B, 300, 130, 0, np.int16, 15, seed=77)
    import torch
    L = got.shape[1]
    out = torch.empty((L, 8), dtype=torch.int32, device="cuda")
    B.fr_export(B.fr_vec(got.cuda(), L), L, out)
    torch.cuda.synchronize()
    w = out.cpu().numpy().astype(np.uint32).astype(object)
    vals = [sum(int(w[i, j]) << (32 * j) for j in range(8)) for i in range(L)]
    assert vals == oracle.partial_eval_rows(M, pt)


def test_noalloc_refuses_shapes_beyond_its_scratch(B):
    # refused on the host before any device work (the pointers are never read)
    L = B.lib()
    rows, cols = 1 << 20, 1024
    assert B.partial_eval_workspace_size(rows, cols, 0, np.int16) > B.NOALLOC_SCRATCH_BYTES
    eq = B.vl_fr_vec(0x1000, 1 << 20, 1 << 20)
    out = B.vl_fr_vec(0x2000, cols, cols)
    st = L.vl_mle_partial_eval_noalloc(ctypes.c_void_p(0x3000), B.VL_I16, rows, cols, cols, 0, eq, out, None, None)
    assert st == B.VL_ERR_WORKSPACE
    assert "fixed scratch" in B.last_error()
