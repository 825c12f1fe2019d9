"""Pins of the Hyrax commitment oracle (oracle/hyrax.py) against facts fixed outside it (no GPU).

  * the base field: q prime, q = 3 mod 4, 381 bits, and the scalar field of
    the proofs equal to the curve's group order r = x^4 - x^2 + 1 of the same
    BLS12 parameter x;
  * the published generator lies on y^2 = x^3 + 4 and has order r;
  * the group law: identity, inverses, commutativity, associativity,
    doubling, and scalar multiplication distributing over addition;
  * hashed generators lie on the curve, in the order-r subgroup, distinct;
  * commitments are additively homomorphic, a single entry commits to its
    scalar multiple of its generator, and small entries agree with repeated
    addition;
  * an opening returns the matrix MLE value and every tamper is rejected;
  * point encoding round-trips and rejects points off the curve.
"""
import random

import numpy as np
import pytest

import oracle.hyrax as hy
from oracle import P as R_ORDER, matrix_mle
from oracle.mle import num_vars


def _probable_prime(n: int, rounds: int = 20) -> bool:
    if n < 2:
        return False
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    rng = random.Random(n & 0xffff)
    for _ in range(rounds):
        a = rng.randrange(2, n - 1)
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def test_base_field_and_group_order():
    assert _probable_prime(hy.Q) and hy.Q % 4 == 3 and hy.Q.bit_length() == 381
    x = hy.BLS_X
    assert R_ORDER == x ** 4 - x ** 2 + 1
    assert _probable_prime(R_ORDER)
    assert hy.H_EFF == 0xd201000000010001


def test_published_generator_has_order_r():
    assert hy.on_curve(hy.G1)
    assert hy.mul(R_ORDER, hy.G1) is None
    assert hy.mul(R_ORDER - 1, hy.G1) == hy.neg(hy.G1)
    assert hy.mul(2, hy.G1) is not None


def test_group_law():
    rng = random.Random(5)
    Ps = [hy.mul(rng.randrange(1, R_ORDER), hy.G1) for _ in range(3)]
    a, b, c = Ps
    assert hy.add(a, None) == a and hy.add(None, a) == a
    assert hy.add(a, hy.neg(a)) is None
    assert hy.add(a, b) == hy.add(b, a)
    assert hy.add(hy.add(a, b), c) == hy.add(a, hy.add(b, c))
    assert hy.add(a, a) == hy.mul(2, a)
    k1, k2 = rng.randrange(R_ORDER), rng.randrange(R_ORDER)
    assert hy.mul(k1 + k2, a) == hy.add(hy.mul(k1, a), hy.mul(k2, a))
    assert hy.mul(-k1, a) == hy.neg(hy.mul(k1, a))
    for Pt in Ps:
        assert hy.on_curve(Pt)


def test_hashed_generators_are_in_the_subgroup():
    gens = hy.generators(6)
    assert len(set(gens)) == 6
    for G in gens:
        assert G is not None and hy.on_curve(G)
        assert hy.mul(R_ORDER, G) is None


def test_cofactor_clearing_is_needed_and_sufficient():
    # a point of the whole curve group is in general outside the order-r
    # subgroup; h_eff times it is inside
    ctr = 0
    while True:
        X = (12345 + ctr) % hy.Q
        s = (X ** 3 + hy.B_COEF) % hy.Q
        if pow(s, (hy.Q - 1) // 2, hy.Q) == 1:
            break
        ctr += 1
    Pt = (X, pow(s, (hy.Q + 1) // 4, hy.Q))
    assert hy.on_curve(Pt)
    assert hy.mul(R_ORDER, Pt) is not None
    assert hy.mul(R_ORDER, hy.mul(hy.H_EFF, Pt)) is None


def _rand_matrix(seed, R, m, lo=-(1 << 15), hi=(1 << 15)):
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi, size=(R, m)).astype(np.int64)


def test_commitments_are_homomorphic():
    gens = hy.generators(5)
    M1, M2 = _rand_matrix(1, 3, 5), _rand_matrix(2, 3, 5)
    C1, C2, C12 = hy.commit(M1, gens), hy.commit(M2, gens), hy.commit(M1 + M2, gens)
    for a, b, ab in zip(C1, C2, C12):
        assert hy.add(a, b) == ab
    Cn = hy.commit(-M1, gens)
    for a, n in zip(C1, Cn):
        assert hy.neg(a) == n


def test_single_entry_and_repeated_addition():
    gens = hy.generators(4)
    M = np.zeros((2, 4), dtype=np.int64)
    M[1, 2] = -7
    C = hy.commit(M, gens)
    assert C[0] is None
    acc = None
    for _ in range(7):
        acc = hy.add(acc, gens[2])
    assert C[1] == hy.neg(acc)
    M = np.array([[3, 1, 0, 2]], dtype=np.int64)
    acc = None
    for v, G in zip(M[0], gens):
        for _ in range(int(v)):
            acc = hy.add(acc, G)
    assert hy.commit(M, gens)[0] == acc


@pytest.mark.parametrize("R,m", [(4, 8), (3, 5), (1, 4), (8, 1)])
def test_opening_is_complete_and_sound(R, m):
    gens = hy.generators(m)
    M = _rand_matrix(R * 10 + m, R, m)
    C = hy.commit(M, gens)
    rng = random.Random(R + m)
    x = [rng.randrange(R_ORDER) for _ in range(num_vars(R))]
    y = [rng.randrange(R_ORDER) for _ in range(num_vars(m))]
    w = hy.open_at(M, x)
    assert hy.verify_open(C, gens, x, y, w) == matrix_mle(M, x, y)
    for j in range(m):
        bad = list(w)
        bad[j] = (bad[j] + 1) % R_ORDER
        with pytest.raises(ValueError):
            hy.verify_open(C, gens, x, y, bad)
    Cb = list(C)
    Cb[0] = hy.add(Cb[0], gens[0])
    with pytest.raises(ValueError):
        hy.verify_open(Cb, gens, x, y, w)


def test_encoding_round_trip():
    G = hy.generator(3)
    assert hy.decode(hy.encode(G)) == G
    assert hy.decode(hy.encode(None)) is None
    bad = bytearray(hy.encode(G))
    bad[50] ^= 1
    with pytest.raises(ValueError):
        hy.decode(bytes(bad))
