"""Hyrax commitments to matrix MLEs (oracle; test infrastructure).

The paper commits to the tensors of a LoRA step with Hyrax (Sec. II-A,
polynomial commitments; Sec. V; Table t2 reports the commitment times and
sizes, which dominate its wall clock).  For a multilinear polynomial given by
the R x m matrix M of its evaluations (rows indexed by the first log R
variables), the commitment is one Pedersen vector commitment per row,

    C_i = sum_j M[i, j] G_j        (i < R),

over fixed generators G_0 .. G_{m-1} of a group where discrete logarithms
are hard.  To open M~(x, y), the prover sends w = sum_i eq(x, i) M[i, .];
the verifier checks sum_j w_j G_j = sum_i eq(x, i) C_i (the commitments are
additively homomorphic) and computes the value sum_j w_j eq(y, j).

Readings and choices (the paper names Hyrax, not its parameters):
  * the group is G1 of BLS12-381, whose order is the scalar field Fr of the
    proofs (p below); the base field Fq, the curve y^2 = x^3 + 4 and the
    generator are the curve's published ones, and Fq is pinned to the BLS12
    parameterisation q = (x - 1)^2 (x^4 - x^2 + 1) / 3 + x;
  * generators by try-and-increment hashing to the curve: for ctr = 0, 1, ..
    X = LE(H(tag || u32 j || u32 ctr || 0) || H(tag || u32 j || u32 ctr || 1))
    mod q, accepted when X^3 + 4 is a square; y = (X^3 + 4)^((q + 1) / 4)
    (q = 3 mod 4), the even root taken; G_j = h_eff (X, y) with the
    effective cofactor h_eff = 1 - x = 0xd201000000010001, so G_j lies in the
    order-p subgroup and nobody knows a relation between the G_j;
    tag = "VeriLoRA-hyrax-v1", H = SHA-256;
  * commitments are not hiding (the blinding term of zero-knowledge Hyrax is
    part of the zero-knowledge masking, out of scope);
  * a point is encoded as 96 bytes, X then Y, each 48 bytes little-endian
    canonical; the point at infinity as 96 zero bytes.
"""
import hashlib
import struct
from typing import List, Optional, Sequence, Tuple

from .field import P as R_ORDER
from .mle import eq_table, partial_eval_rows

BLS_X = -0xd201000000010000
Q = (BLS_X - 1) ** 2 * (BLS_X ** 4 - BLS_X ** 2 + 1) // 3 + BLS_X
B_COEF = 4
H_EFF = 1 - BLS_X
G1 = (0x17f1d3a73197d7942695638c4fa9ac0fc3688c4f9774b905a14e3a3f171bac586c55e83ff97a1aeffb3af00adb22c6bb,
      0x08b3f481e3aaa0f1a09e30ed741d8ae4fcf5e095d5d00af600db18cb2c04b3edd03cc744a2888ae40caa232946c5e7e1)
TAG = b"VeriLoRA-hyrax-v1"

Point = Optional[Tuple[int, int]]   # affine, None = infinity


def on_curve(Pt: Point) -> bool:
    if Pt is None:
        return True
    x, y = Pt
    return (y * y - x * x * x - B_COEF) % Q == 0


def neg(Pt: Point) -> Point:
    return None if Pt is None else (Pt[0], (-Pt[1]) % Q)


def add(P1: Point, P2: Point) -> Point:
    """Affine addition on y^2 = x^3 + 4 (chord and tangent)."""
    if P1 is None:
        return P2
    if P2 is None:
        return P1
    x1, y1 = P1
    x2, y2 = P2
    if x1 == x2:
        if (y1 + y2) % Q == 0:
            return None
        lam = 3 * x1 * x1 * pow(2 * y1, -1, Q) % Q
    else:
        lam = (y2 - y1) * pow(x2 - x1, -1, Q) % Q
    x3 = (lam * lam - x1 - x2) % Q
    y3 = (lam * (x1 - x3) - y1) % Q
    return (x3, y3)


def mul(k: int, Pt: Point) -> Point:
    """k P by double-and-add (k any integer; negative k negates)."""
    if k < 0:
        return mul(-k, neg(Pt))
    acc: Point = None
    addend = Pt
    while k:
        if k & 1:
            acc = add(acc, addend)
        addend = add(addend, addend)
        k >>= 1
    return acc


def encode(Pt: Point) -> bytes:
    if Pt is None:
        return bytes(96)
    return Pt[0].to_bytes(48, "little") + Pt[1].to_bytes(48, "little")


def decode(b: bytes) -> Point:
    if len(b) != 96:
        raise ValueError("a point is 96 bytes")
    if b == bytes(96):
        return None
    x, y = int.from_bytes(b[:48], "little"), int.from_bytes(b[48:], "little")
    if x >= Q or y >= Q or not on_curve((x, y)):
        raise ValueError("not a canonical point of the curve")
    return (x, y)


def _h(data: bytes) -> bytes:
    return hashlib.sha256(data).digest()


def generator(j: int) -> Tuple[int, int]:
    """G_j by try-and-increment hashing to the curve, then cofactor clearing."""
    ctr = 0
    while True:
        pre = TAG + struct.pack("<II", j, ctr)
        X = int.from_bytes(_h(pre + b"\x00") + _h(pre + b"\x01"), "little") % Q
        s = (X * X * X + B_COEF) % Q
        if pow(s, (Q - 1) // 2, Q) == 1:
            y = pow(s, (Q + 1) // 4, Q)
            if y & 1:
                y = Q - y
            G = mul(H_EFF, (X, y))
            if G is not None:
                return G
        ctr += 1


def generators(m: int) -> List[Tuple[int, int]]:
    return [generator(j) for j in range(m)]


def commit(M, gens: Sequence[Point]) -> List[Point]:
    """C_i = sum_j M[i, j] G_j for every row i (integer entries)."""
    out = []
    for row in M:
        acc: Point = None
        for v, G in zip(row, gens):
            acc = add(acc, mul(int(v), G))
        out.append(acc)
    return out


def open_at(M, x: Sequence[int]) -> List[int]:
    """w = sum_i eq(x, i) M[i, .] (the prover's opening message for any y)."""
    import numpy as np
    return partial_eval_rows(np.asarray(M), x)


def verify_open(commits: Sequence[Point], gens: Sequence[Point], x: Sequence[int], y: Sequence[int],
                w: Sequence[int]) -> int:
    """Checks sum_j w_j G_j = sum_i eq(x, i) C_i and returns the value
    sum_j w_j eq(y, j); raises ValueError on a failed check."""
    ex, ey = eq_table(x), eq_table(y)
    lhs: Point = None
    for wj, G in zip(w, gens):
        lhs = add(lhs, mul(wj % R_ORDER, G))
    rhs: Point = None
    for ei, C in zip(ex, commits):
        rhs = add(rhs, mul(ei, C))
    if lhs != rhs:
        raise ValueError("opening does not match the commitments")
    return sum(wj * ej for wj, ej in zip(w, ey)) % R_ORDER
