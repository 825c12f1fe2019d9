"""Multilinear extensions, written from the definition (oracle; test infrastructure).

eq. (MLE), Sec. II-B.2: for f on {0,1}^n,
    f~(x) = sum_{b in {0,1}^n} f(b) * prod_i (b_i x_i + (1 - b_i)(1 - x_i)).
A matrix with D0 x D1 entries is read as a function on {0,1}^{n0} x {0,1}^{n1}
after zero padding every dimension to a power of two (Sec. II-C).

Index-to-bits order (the paper leaves it open): b_1 is the most significant
bit of the index, so that index i of a length-2^n vector is the bit string
(b_1, ..., b_n) read as a binary number.
"""
from typing import List, Sequence

import numpy as np

from .field import P


def num_vars(d: int) -> int:
    """Smallest n with 2^n >= d (a dimension of size 1 has no variables)."""
    if d < 1:
        raise ValueError("dimension must be >= 1")
    n = 0
    while (1 << n) < d:
        n += 1
    return n


def bits_msb_first(i: int, n: int) -> List[int]:
    return [(i >> (n - 1 - j)) & 1 for j in range(n)]


def eq_basis(x: Sequence[int], b: Sequence[int]) -> int:
    """prod_i (b_i x_i + (1 - b_i)(1 - x_i)) mod p  -- the Lagrange basis of eq. (MLE)."""
    assert len(x) == len(b)
    out = 1
    for xi, bi in zip(x, b):
        out = out * (bi * xi + (1 - bi) * (1 - xi)) % P
    return out


def eq_table(x: Sequence[int]) -> List[int]:
    """eq_basis(x, bits(i)) for every index i in [0, 2^n)."""
    n = len(x)
    return [eq_basis(x, bits_msb_first(i, n)) for i in range(1 << n)]


def mle_eval(values: Sequence[int], x: Sequence[int]) -> int:
    """f~(x) for f given by its values at indices 0..len-1 (zero beyond)."""
    n = len(x)
    assert len(values) <= (1 << n)
    total = 0
    for i, fv in enumerate(values):
        total += int(fv) * eq_basis(x, bits_msb_first(i, n))
    return total % P


def matrix_mle(M: np.ndarray, x: Sequence[int], y: Sequence[int]) -> int:
    """M~(x, y) = sum_{i,k} M[i,k] eq(x, i) eq(y, k)  (rows first, then columns)."""
    d0, d1 = M.shape
    assert num_vars(d0) == len(x) and num_vars(d1) == len(y)
    ex = eq_table(x)
    ey = eq_table(y)
    total = 0
    for i in range(d0):
        for k in range(d1):
            total += int(M[i, k]) * ex[i] * ey[k]
    return total % P


def partial_eval_rows(M: np.ndarray, x: Sequence[int]) -> List[int]:
    """a[k] = M~(x, k) = sum_i eq(x, i) M[i, k] for every k < 2^{n1} (zero padded)."""
    d0, d1 = M.shape
    assert num_vars(d0) == len(x)
    ex = eq_table(x)
    acc = np.zeros(d1, dtype=object)
    for i in range(d0):
        acc = acc + ex[i] * M[i, :].astype(object)
    out = [int(v) % P for v in acc]
    return out + [0] * ((1 << num_vars(d1)) - d1)


def partial_eval_cols(M: np.ndarray, y: Sequence[int]) -> List[int]:
    """b[k] = M~(k, y) = sum_j M[k, j] eq(y, j) for every k < 2^{n0} (zero padded)."""
    d0, d1 = M.shape
    assert num_vars(d1) == len(y)
    ey = eq_table(y)
    acc = np.zeros(d0, dtype=object)
    for j in range(d1):
        acc = acc + M[:, j].astype(object) * ey[j]
    out = [int(v) % P for v in acc]
    return out + [0] * ((1 << num_vars(d0)) - d0)
