"""Lookup argument, prover and verifier (oracle; test infrastructure).

Protocol 1 (Sec. II-D) proves that every entry s_i of a secret vector S
(length D) lies in a public table T (length N): with m_j the number of i with
s_i = t_j, the logarithmic derivatives of prod (X + s_i) and
prod (X + t_j)^{m_j} agree (eq. (rational-function)), which at a random
beta is sum_i A_i = sum_j m_j B_j for A_i = 1/(beta + s_i), B_j = 1/(beta + t_j).
With a further random alpha and a random point u, eq. (lookup-sumcheck)
folds this and the two inverse relations into one sum over the D indices
x = (x_H, x_L) (x_H the top log(D/N) bits, x_L the low log N bits):

    alpha + alpha^2 = sum_x [ alpha A(x) eq(u, x) (S(x) + beta) + A(x)
                              + (N/D) alpha^2 B(x_L) eq(u_L, x_L) (T(x_L) + beta)
                              - (N/D) B(x_L) m(x_L) ],

u_L the last log N coordinates of u.  On the Boolean hypercube
A (S + beta) = 1 and B (T + beta) = 1, so the first and third terms add up to
alpha and alpha^2 (eq(u, .) sums to 1) and the second and fourth cancel
exactly when sum_i A_i = sum_j m_j B_j.  The sumcheck over x (most
significant bit first) has rounds of degree 3, sent as g(0..3); it ends with
the values A(r), S(r), B(r_L), T(r_L), m(r_L), which the openings of the
committed tensors would check (Sec. II-A; here a witness check stands in).

Readings (the paper's equation is garbled in places):
  * "i (+) j" is the concatenation of the index bits, i in [D/N] high;
    \\widetilde{e}(u, .) is the eq polynomial of eq. (MLE);
  * D and N are powers of two with N | D: S is padded to a power of two
    (at least N) with the table's first entry, which keeps S in T and is
    counted by m;
  * tables are ranges of consecutive integers t_j = t0 + j, optionally with a
    second column (compressed as t_j = (t0 + j) + gamma b_j, and
    s_i = x_i + gamma y_i, with gamma squeezed first), the form of the
    paper's tables (F_B ranges, residue ranges, input/output pairs of
    zkSwiGLU and zkSoftmax);
  * transcript: st = H("VeriLoRA-lookup-v1" || u64 seed || u32 id ||
    u64 D || u32 N || i32 t0 || u32 two_col); squeezes "gamma" (two-column
    only), "beta", "alpha", "u" (log D' times, D' the padded length);
    absorbs "round" (g(0..3), then squeezes "r") and "final"
    (A(r), S(r), B(r_L), T(r_L), m(r_L)).  The claimed sum alpha + alpha^2
    is not sent.

Proof bytes: (g0, g1, g2, g3) per round || A(r) || S(r) || B(r_L) || T(r_L)
|| m(r_L), 32-byte canonical little-endian field elements.
"""
import struct
from typing import List, Optional, Sequence

import numpy as np

from .field import P, enc, dec, inv
from .mle import eq_table, eq_basis, mle_eval
from .transcript import Transcript, sha256
from .zkmat import FalseStatement, Reject

DOMAIN = b"VeriLoRA-lookup-v1"


def padded_len(D: int, N: int) -> int:
    n = max(N, 1)
    while n < D:
        n *= 2
    return n


def log2(n: int) -> int:
    k = 0
    while (1 << k) < n:
        k += 1
    assert (1 << k) == n, "not a power of two"
    return k


def transcript(seed: int, lid: int, D: int, N: int, t0: int, two_col: bool) -> Transcript:
    return Transcript.from_state(sha256(DOMAIN + struct.pack("<QIQIiI", seed, lid, D, N, t0, int(two_col))))


def challenges(tr: Transcript, n: int, two_col: bool):
    gamma = tr.squeeze(b"gamma") if two_col else 0
    beta = tr.squeeze(b"beta")
    alpha = tr.squeeze(b"alpha")
    u = [tr.squeeze(b"u") for _ in range(n)]
    return gamma, beta, alpha, u


def multiplicities(xs: Sequence[int], ys: Optional[Sequence[int]], t0: int, tb: Optional[Sequence[int]],
                   N: int) -> List[int]:
    """m_j = |{i : (x_i, y_i) = (t0 + j, tb_j)}| (pairs compared as integers);
    raises FalseStatement if some entry is not in the table."""
    where = {}
    for j in range(N):
        where[(t0 + j, tb[j] if tb is not None else 0)] = j
    m = [0] * N
    for i, x in enumerate(xs):
        key = (int(x), int(ys[i]) if ys is not None else 0)
        if key not in where:
            raise FalseStatement(f"entry {i} = {key} is not in the table")
        m[where[key]] += 1
    return m


def _line(x, h: int, X: int):
    """x_t + X (x_{t+h} - x_t) for t < h (numpy object arrays of Python ints)."""
    return (x[:h] + X * (x[h:2 * h] - x[:h])) % P


def _sum_terms(terms, h: int, X: int) -> int:
    """sum over t < h of sum over terms coef * prod of the tables' lines at X"""
    total = 0
    for coef, tabs in terms:
        prod = None
        for tb in tabs:
            ln = _line(tb, h, X)
            prod = ln if prod is None else prod * ln % P
        total += coef * int(prod.sum())
    return total % P


def _obj(v):
    return np.array([int(x) % P for x in v], dtype=object)


def _setup(xs, ys, t0, tb, N, seed, lid):
    D = len(xs)
    two = ys is not None
    Dp = padded_len(D, N)
    n, nL = log2(Dp), log2(N)
    nH = n - nL
    pad = Dp - D
    xs_p = [int(x) for x in xs] + [t0] * pad
    ys_p = ([int(y) for y in ys] + [int(tb[0])] * pad) if two else None
    tr = transcript(seed, lid, D, N, t0, two)
    gamma, beta, alpha, u = challenges(tr, n, two)
    S = [(xs_p[i] + gamma * (ys_p[i] if two else 0)) % P for i in range(Dp)]
    T = [(t0 + j + gamma * (int(tb[j]) if two else 0)) % P for j in range(N)]
    return dict(D=D, Dp=Dp, n=n, nL=nL, nH=nH, xs=xs_p, ys=ys_p, tr=tr, gamma=gamma, beta=beta, alpha=alpha,
                u=u, S=S, T=T)


def prove(xs: Sequence[int], ys: Optional[Sequence[int]], t0: int, tb: Optional[Sequence[int]], N: int,
          seed: int, lid: int, m_override: Optional[List[int]] = None):
    """Prove that every (x_i[, y_i]) is a row of the table ((t0 + j[, tb_j]),
    j < N).  Returns (proof bytes, final transcript state, details).
    ``m_override`` replaces the multiplicities (tests of a cheating prover)."""
    st = _setup(xs, ys, t0, tb, N, seed, lid)
    Dp, n, nL, nH = st["Dp"], st["n"], st["nL"], st["nH"]
    tr, beta, alpha, u = st["tr"], st["beta"], st["alpha"], st["u"]
    m = multiplicities(st["xs"], st["ys"], t0, tb, N) if m_override is None else list(m_override)

    Sb = [(s + beta) % P for s in st["S"]]
    Tb = [(t + beta) % P for t in st["T"]]
    if any(v == 0 for v in Sb) or any(v == 0 for v in Tb):
        raise FalseStatement("beta hits a pole of the rational function")
    A = [inv(v) for v in Sb]
    Bt = [inv(v) for v in Tb]
    E = eq_table(u)
    EL = eq_table(u[nH:])
    c2 = N * inv(Dp) % P
    c1 = c2 * alpha % P * alpha % P
    # the tables of the low index x_L repeated over the high index
    Bx = [Bt[i % N] for i in range(Dp)]
    ELx = [EL[i % N] for i in range(Dp)]
    Tx = [Tb[i % N] for i in range(Dp)]
    mx = [m[i % N] % P for i in range(Dp)]
    terms = [(alpha, [E, A, Sb]), (1, [A]), (c1, [Bx, ELx, Tx]), ((P - c2) % P, [Bx, mx])]
    claim = (alpha + alpha * alpha) % P
    if sum(c * _prod_sum(tabs) for c, tabs in terms) % P != claim:
        raise FalseStatement("the lookup sum differs from alpha + alpha^2")
    terms = [(c, [_obj(tb_) for tb_ in tabs]) for c, tabs in terms]

    rounds, rs = [], []
    for rd in range(n):
        h = len(terms[0][1][0]) // 2
        g = [_sum_terms(terms, h, X) for X in range(4)]
        tr.absorb(b"round", b"".join(enc(x) for x in g))
        r = tr.squeeze(b"r")
        terms = [(c, [_line(tb_, h, r) for tb_ in tabs]) for c, tabs in terms]
        rounds.append(g)
        rs.append(r)
    E_, A_, Sb_ = terms[0][1]
    Bx_, ELx_, Tx_ = terms[2][1]
    mx_ = terms[3][1][1]
    fin = [int(A_[0]), int(Sb_[0] - beta) % P, int(Bx_[0]), int(Tx_[0] - beta) % P, int(mx_[0])]
    tr.absorb(b"final", b"".join(enc(v) for v in fin))
    proof = b"".join(enc(x) for g in rounds for x in g) + b"".join(enc(v) for v in fin)
    details = dict(gamma=st["gamma"], beta=beta, alpha=alpha, u=u, r=rs, rounds=rounds, finals=fin, m=m,
                   Dp=Dp, nH=nH, nL=nL)
    return proof, tr.state, details


def _prod_sum(tabs) -> int:
    s = 0
    for t in range(len(tabs[0])):
        p = 1
        for tb in tabs:
            p = p * tb[t] % P
        s += p
    return s % P


def proof_len(D: int, N: int) -> int:
    return 32 * (4 * log2(padded_len(D, N)) + 5)


def verify(proof: bytes, D: int, N: int, t0: int, two_col: bool, seed: int, lid: int,
           witness: Optional[tuple] = None):
    """Check a proof; returns the reduced claims, raises Reject.

    Without a witness this checks the sumcheck of eq. (lookup-sumcheck):
    g(0) + g(1) equals the running claim (alpha + alpha^2 at the start), the
    claim moves to g(r) by cubic interpolation, and the last claim equals the
    summand at r from the sent values A(r), S(r), B(r_L), T(r_L), m(r_L).
    With a witness (xs, ys, tb) it also checks those five values by direct
    evaluation of the multilinear extensions of the padded S, of T, of the
    multiplicities and of the inverses (standing in for the openings of the
    committed tensors, which are out of scope)."""
    from .bmm import lagrange_eval
    Dp = padded_len(D, N)
    n, nL = log2(Dp), log2(N)
    nH = n - nL
    if len(proof) != proof_len(D, N):
        raise Reject("length")
    try:
        el = [dec(proof[i:i + 32]) for i in range(0, len(proof), 32)]
    except ValueError:
        raise Reject("encoding")
    tr = transcript(seed, lid, D, N, t0, two_col)
    gamma, beta, alpha, u = challenges(tr, n, two_col)
    claim = (alpha + alpha * alpha) % P
    rs = []
    for rd in range(n):
        g = el[4 * rd:4 * rd + 4]
        if (g[0] + g[1]) % P != claim:
            raise Reject("round", rd + 1)
        tr.absorb(b"round", b"".join(enc(x) for x in g))
        r = tr.squeeze(b"r")
        claim = lagrange_eval(g, r)
        rs.append(r)
    Av, Sv, Bv, Tv, mv = el[4 * n:4 * n + 5]
    rL = rs[nH:]
    c2 = N * inv(Dp) % P
    c1 = c2 * alpha % P * alpha % P
    expect = (alpha * Av % P * eq_basis(u, rs) % P * (Sv + beta) + Av
              + c1 * Bv % P * eq_basis(u[nH:], rL) % P * (Tv + beta) - c2 * Bv % P * mv) % P
    if expect != claim:
        raise Reject("final", n)
    tr.absorb(b"final", b"".join(enc(v) for v in (Av, Sv, Bv, Tv, mv)))
    if witness is not None:
        xs, ys, tb = witness
        st = _setup(xs, ys, t0, tb, N, seed, lid)
        m = multiplicities(st["xs"], st["ys"], t0, tb, N)
        if mle_eval(st["S"], rs) != Sv or mle_eval(st["T"], rL) != Tv or mle_eval(m, rL) != mv:
            raise Reject("witness")
        if mle_eval([inv((s + beta) % P) for s in st["S"]], rs) != Av:
            raise Reject("witness")
        if mle_eval([inv((t + beta) % P) for t in st["T"]], rL) != Bv:
            raise Reject("witness")
    return dict(gamma=gamma, beta=beta, alpha=alpha, u=u, r=rs, finals=[Av, Sv, Bv, Tv, mv], state=tr.state)


def prove_case(lk, seed: int):
    """Convenience: prove a ``workloads.LookupCase``."""
    return prove(lk.x.tolist(), lk.y.tolist() if lk.y is not None else None, lk.t0,
                 lk.tb.tolist() if lk.tb is not None else None, lk.N, seed, lk.lid)
