"""Batched (per-head) matmul sumcheck, prover and verifier (oracle; test infrastructure).

Multi-head attention (Sec. III-A, eq. (att)) multiplies one pair of matrices
per head: S_h = Q_h K_h^T and O_h = P_h V_h for h < H, and its backward pass
does the same with dO, dS.  Each head's product is the statement of
eq. (matmul); this module proves all H of them with one sumcheck by treating
the head index as H's own variables.  With the head dimension zero padded to
2^{nh} like every other dimension (Sec. II-C), the 3-D tensor C[h, i, j] has
the multilinear extension of eq. (MLE) over (h, i, j), and C_h = A_h B_h for
every h iff, for random rho, u, v,

    C~(rho, u, v) = sum_{h in {0,1}^nh} sum_{w in {0,1}^n1}
                        eq(rho, h) * A~(h, u, w) * B~(h, w, v)

(the multilinear extension in h of sum_w A~(h,u,w) B~(h,w,v), evaluated at
rho by eq. (MLE)).  The sum runs over the nh + n1 variables (h, w), head
variables first, each most significant first.  In a head round the summand
is a product of three multilinear functions of the round's variable, so the
round polynomial has degree 3 and is sent as g(0), g(1), g(2), g(3); after
the head rounds eq(rho, r_h) is one number and the w rounds have degree 2
(g(0), g(1), g(2)), as in the plain matmul sumcheck.  The last claim must be
eq(rho, r_h) * A~(r_h, u, r_w) * B~(r_h, r_w, v).

Readings (the paper gives the attention formula, not its proof):
  * the head index is the most significant index of the 3-D tensors, and
    rho is squeezed before u and v;
  * transcript: st = H("VeriLoRA-zkBMat-v1" || u64 seed || u32 group_id ||
    u32 H || u32 D0 || u32 D1 || u32 D2); squeezes "h" (nh times), "u" (n0),
    "v" (n2); absorbs "claim" c, "round" (the 4 or 3 values of each round),
    "final" (a_final || b_final); each round's challenge is squeezed with "r".

Proof bytes: c || (g0, g1, g2, g3) per head round || (g0, g1, g2) per w round
|| a_final || b_final, 32-byte canonical little-endian field elements.
"""
import struct
from typing import List, Optional, Sequence

import numpy as np

from .field import P, enc, dec, inv
from .mle import num_vars, eq_table, eq_basis, bits_msb_first, partial_eval_rows, partial_eval_cols
from .transcript import Transcript, sha256
from .zkmat import FalseStatement, Reject

DOMAIN = b"VeriLoRA-zkBMat-v1"


def transcript(seed: int, group_id: int, H: int, d0: int, d1: int, d2: int) -> Transcript:
    return Transcript.from_state(sha256(DOMAIN + struct.pack("<QIIIII", seed, group_id, H, d0, d1, d2)))


def challenges(tr: Transcript, H: int, d0: int, d2: int):
    rho = [tr.squeeze(b"h") for _ in range(num_vars(H))]
    u = [tr.squeeze(b"u") for _ in range(num_vars(d0))]
    v = [tr.squeeze(b"v") for _ in range(num_vars(d2))]
    return rho, u, v


def tensor_mle(Ms: Sequence[np.ndarray], h: Sequence[int], x: Sequence[int], y: Sequence[int]) -> int:
    """M~(h, x, y) of the 3-D tensor M[k, i, j] = Ms[k][i, j] (zero padded in
    every index) by eq. (MLE): sum over (k, i, j) of M[k, i, j] times
    eq(h, k) eq(x, i) eq(y, j)."""
    nh = len(h)
    assert len(Ms) <= (1 << nh)
    ex = eq_table(x)
    ey = eq_table(y)
    total = 0
    for k, M in enumerate(Ms):
        ek = eq_basis(h, bits_msb_first(k, nh))
        d0, d1 = M.shape
        for i in range(d0):
            for j in range(d1):
                total += ek * ex[i] * ey[j] * int(M[i, j])
    return total % P


def claim_value(Cs: Sequence[np.ndarray], rho: Sequence[int], u: Sequence[int], v: Sequence[int]) -> int:
    """c = C~(rho, u, v) summed in the order heads, rows, columns:
    sum_k eq(rho, k) sum_i eq(u, i) sum_j C_k[i, j] eq(v, j) (the same value as
    tensor_mle; the inner sums run over numpy rows, for full-size tensors)."""
    er, eu = eq_table(rho), eq_table(u)
    total = 0
    for k, C in enumerate(Cs):
        t = partial_eval_cols(C, v)
        total += er[k] * (sum(eu[i] * t[i] for i in range(len(t))) % P)
    return total % P


def lagrange_eval(gs: Sequence[int], r: int) -> int:
    """The polynomial of degree len(gs) - 1 through (k, gs[k]), k = 0.., at r."""
    n = len(gs)
    total = 0
    for k in range(n):
        num, den = 1, 1
        for m in range(n):
            if m != k:
                num = num * (r - m) % P
                den = den * (k - m) % P
        total += gs[k] * num * inv(den)
    return total % P


def proof_len(H: int, d1: int) -> int:
    return 32 * (1 + 4 * num_vars(H) + 3 * num_vars(d1) + 2)


def _line(x: Sequence[int], h: int, X: int) -> List[int]:
    """x_t + X (x_{t+h} - x_t) for t < h: the table restricted to X in the
    leading variable."""
    return [(x[t] + X * (x[t + h] - x[t])) % P for t in range(h)]


def prove(As: Sequence[np.ndarray], Bs: Sequence[np.ndarray], Cs: Sequence[np.ndarray], seed: int,
          group_id: int):
    """Prove C_h = A_h B_h for every head h (A_h D0 x D1, B_h D1 x D2, C_h
    D0 x D2, integer arrays, transposed views already applied).

    Returns (proof bytes, final transcript state, details).  Raises
    FalseStatement if the sum of eq(rho, h) A~ B~ differs from C~(rho, u, v).
    """
    H = len(As)
    assert H >= 1 and len(Bs) == H and len(Cs) == H
    d0, d1 = As[0].shape
    d2 = Bs[0].shape[1]
    for A, B, C in zip(As, Bs, Cs):
        assert A.shape == (d0, d1) and B.shape == (d1, d2) and C.shape == (d0, d2)
    nh, n1 = num_vars(H), num_vars(d1)
    L1 = 1 << n1

    tr = transcript(seed, group_id, H, d0, d1, d2)
    rho, u, v = challenges(tr, H, d0, d2)
    c = claim_value(Cs, rho, u, v)
    tr.absorb(b"claim", enc(c))

    # tables over (h, w), head index most significant; padding heads are zero
    E, a, b = [], [], []
    erho = eq_table(rho)
    for k in range(1 << nh):
        E += [erho[k]] * L1
        if k < H:
            a += partial_eval_rows(As[k], u)     # A~(k, u, w)
            b += partial_eval_cols(Bs[k], v)     # B~(k, w, v)
        else:
            a += [0] * L1
            b += [0] * L1
    if sum(e * x * y for e, x, y in zip(E, a, b)) % P != c:
        raise FalseStatement("sum of eq(rho,h) A~(h,u,w) B~(h,w,v) differs from C~(rho,u,v)")

    rounds, rs = [], []
    for rd in range(nh + n1):
        half = len(a) // 2
        deg = 3 if rd < nh else 2
        g = []
        for X in range(deg + 1):
            eX, aX, bX = _line(E, half, X), _line(a, half, X), _line(b, half, X)
            g.append(sum(p * q * s for p, q, s in zip(eX, aX, bX)) % P)
        tr.absorb(b"round", b"".join(enc(x) for x in g))
        r = tr.squeeze(b"r")
        E, a, b = _line(E, half, r), _line(a, half, r), _line(b, half, r)
        rounds.append(g)
        rs.append(r)
    tr.absorb(b"final", enc(a[0]) + enc(b[0]))
    proof = enc(c) + b"".join(enc(x) for g in rounds for x in g) + enc(a[0]) + enc(b[0])
    details = dict(rho=rho, u=u, v=v, c=c, r=rs, rounds=rounds, a_final=a[0], b_final=b[0], e_final=E[0])
    return proof, tr.state, details


def verify(proof: bytes, H: int, d0: int, d1: int, d2: int, seed: int, group_id: int,
           witness: Optional[tuple] = None):
    """Check a proof; returns the reduced claims, raises Reject.

    Without a witness this checks the sumcheck: g(0) + g(1) equals the
    running claim each round, the claim moves to g(r) (cubic in a head round,
    quadratic in a w round), and the last claim equals
    eq(rho, r_h) * a_final * b_final.  With a witness (As, Bs, Cs) it also
    checks c = C~(rho, u, v), a_final = A~(r_h, u, r_w) and
    b_final = B~(r_h, r_w, v) by direct evaluation (standing in for the
    commitment openings, which are out of scope)."""
    nh, n1 = num_vars(H), num_vars(d1)
    if len(proof) != proof_len(H, d1):
        raise Reject("length")
    try:
        el = [dec(proof[i:i + 32]) for i in range(0, len(proof), 32)]
    except ValueError:
        raise Reject("encoding")
    tr = transcript(seed, group_id, H, d0, d1, d2)
    rho, u, v = challenges(tr, H, d0, d2)
    c = el[0]
    tr.absorb(b"claim", enc(c))
    claim, pos, rs = c, 1, []
    for rd in range(nh + n1):
        deg = 3 if rd < nh else 2
        g = el[pos:pos + deg + 1]
        pos += deg + 1
        if (g[0] + g[1]) % P != claim:
            raise Reject("round", rd + 1)
        tr.absorb(b"round", b"".join(enc(x) for x in g))
        r = tr.squeeze(b"r")
        claim = lagrange_eval(g, r)
        rs.append(r)
    af, bf = el[pos], el[pos + 1]
    rh, rw = rs[:nh], rs[nh:]
    e = eq_basis(rho, rh)
    if e * af % P * bf % P != claim:
        raise Reject("final", nh + n1)
    tr.absorb(b"final", enc(af) + enc(bf))
    if witness is not None:
        As, Bs, Cs = witness
        if tensor_mle(Cs, rho, u, v) != c:
            raise Reject("witness")
        if tensor_mle(As, rh, u, rw) != af or tensor_mle(Bs, rh, rw, v) != bf:
            raise Reject("witness")
    return dict(rho=rho, u=u, v=v, c=c, r=rs, a_final=af, b_final=bf, state=tr.state)


def prove_batch(bp, seed: int):
    """Convenience: prove a ``workloads.HeadBatch`` (per-head views applied)."""
    return prove(bp.opA_heads(), bp.opB_heads(), bp.C_heads(), seed, bp.group_id)
