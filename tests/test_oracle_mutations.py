"""Planted mistakes in the oracle must be caught by the pins (CPU only).

Each case swaps one oracle function for a plausibly wrong variant (a dropped
term, a wrong sign, a swapped index order, a transposed operand) and checks
that at least one of the independent pins used in test_oracle_pins fails.
"""
import random

import numpy as np
import pytest

import oracle
import oracle.mle as mle
import oracle.zkmat as zk
from oracle import P
import workloads


def _pins_hold() -> bool:
    rng = random.Random(1)
    try:
        # partition of unity and Boolean points
        x = [rng.randrange(P) for _ in range(3)]
        if sum(mle.eq_table(x)) % P != 1:
            return False
        if mle.eq_table([1, 0, 1]) != [1 if i == 5 else 0 for i in range(8)]:
            return False
        # identity closed form through the claim path
        u, v = [rng.randrange(P) for _ in range(2)], [rng.randrange(P) for _ in range(2)]
        expect = 1
        for a, b in zip(u, v):
            expect = expect * (a * b + (1 - a) * (1 - b)) % P
        if zk.claim_value(np.eye(4, dtype=np.int64), u, v) != expect:
            return False
        # completeness with the witness evaluated by definition
        for dims in ([(4, 8, 2)], [(3, 5, 6)], [(2, 4, 2), (2, 2, 2)]):
            g = workloads.tiny_random_group(len(dims) + dims[0][1], dims)
            prods = [(p.opA(), p.opB()) for p in g.products]
            proof, _, _ = zk.prove_group(prods, g.C, 3, 1)
            zk.verify_group(proof, g.shapes, 3, 1, witness=(prods, g.C))
    except (zk.Reject, zk.FalseStatement, AssertionError, ValueError, IndexError):
        return False
    return True


def _eq_basis_dropped_term(x, b):
    out = 1
    for xi, bi in zip(x, b):
        out = out * (bi * xi + (1 - bi)) % P          # lost the (1 - x_i) factor
    return out


def _bits_lsb_first(i, n):
    return [(i >> j) & 1 for j in range(n)]


def _fold_swapped(a, r):
    h = len(a) // 2
    return [(a[t + h] + r * (a[t] - a[t + h])) % P for t in range(h)]


def _round_poly_sign(a, b):
    g0, g1, g2 = _orig_round_poly(a, b)
    h = len(a) // 2
    g2 = sum((2 * a[t + h] + a[t]) * (2 * b[t + h] - b[t]) for t in range(h)) % P
    return g0, g1, g2


def _cols_transposed(M, y):
    return _orig_cols(np.ascontiguousarray(M.T), y) if M.shape[0] == M.shape[1] \
        else _orig_rows(M.T, y)


def _interp_wrong(g0, g1, g2, r):
    return (g0 * (r - 1) * (r - 2) * zk.INV2 + g1 * r * (r - 2) + g2 * r * (r - 1) * zk.INV2) % P


_orig_round_poly = zk.round_poly
_orig_cols = mle.partial_eval_cols
_orig_rows = mle.partial_eval_rows

MUTATIONS = [
    ("eq basis drops (1-x_i)", [(mle, "eq_basis", _eq_basis_dropped_term)]),
    ("LSB-first index bits", [(mle, "bits_msb_first", _bits_lsb_first)]),
    ("fold weights swapped", [(zk, "fold", _fold_swapped)]),
    ("round g(2) sign error", [(zk, "round_poly", _round_poly_sign)]),
    ("cols contraction transposed", [(zk, "partial_eval_cols", _cols_transposed)]),
    ("interpolation sign error", [(zk, "interpolate_quadratic", _interp_wrong)]),
]


def test_unmutated_oracle_passes_the_pins():
    assert _pins_hold()


@pytest.mark.parametrize("name,patches", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, patches, monkeypatch):
    for mod, attr, fn in patches:
        monkeypatch.setattr(mod, attr, fn)
    assert not _pins_hold(), f"pins did not catch: {name}"
