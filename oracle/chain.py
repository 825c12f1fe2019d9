"""One LoRA layer's training step as a chain of claims (oracle; test infrastructure).

The paper proves every matrix product and addition of a LoRA step with zkMat
and composes the steps sequentially (Sec. IV-B, "putting everything
together"): a sumcheck fixes point-value claims, the next step justifies
exactly those points, and the last claims are opened against the committed
tensors.  Protocol 2 proves the parameter update of eq. (grad_update_ab) with
zkMat as well.  This module writes that composition out for one layer
(forward, backward and update of one LoRA target), in one Fiat-Shamir
transcript, as plain Python over the definitions in ``mle`` and ``zkmat``.

Readings taken here (the paper gives the strategy, not the steps):
  * The update A' = A - eta dA is exact over the integers as
        UA = 2^F A - eta dA
    with public integers F (fixed-point scale) and eta (learning rate at scale
    2^-F); UA is the pre-rounding update whose re-quantisation to the next
    step's int16 A is a lookup (out of scope).  Being linear, it holds iff it
    holds for the MLEs at a random point z: UA~(z) = 2^F A~(z) - eta dA~(z).
    The same for B.
  * Matrix additions: the forward output Y = X W + H B and dX = dY W^T + G A^T
    are zkMat sum groups (one transcript branch, part claims).
  * The re-quantised H = requant(X A) and G = requant(dY B^T) are witness
    inputs; the claims the sumchecks leave on them, and the claims on the
    products C2 = X A and C4 = dY B^T that would feed their rounding lookups,
    stay open (lookups are out of scope).
  * The sumchecks of one stage run on forked branches of the transcript,
    H(st || "fork" || k), so that they are independent of each other, and the
    stage ends by absorbing every branch's final state ("join").
  * Several claims M~(x_k, y_k) = v_k on one matrix are reduced to one by a
    random combination and two sumchecks: over the row variables,
        sum_k rho_k v_k = sum_i sum_k rho_k eq(x_k, i) t_k(i),
        t_k(i) = sum_j M[i, j] eq(y_k, j),
    which ends at a row point r with the values t_k(r) = M~(r, y_k); then over
    the column variables,
        sum_k sigma_k t_k(r) = sum_j M~(r, j) sum_k sigma_k eq(y_k, j),
    which ends at one claim M~(r, s).

Transcript (SHA-256, the same absorb / squeeze as ``transcript``):
  init     st = H("VeriLoRA-chain-v1" || u64 seed || u32 T, d_in, d_out, r, F, eta)
  stage 1  squeeze zA (n_in + n_r values, rows first), zB (n_r + n_out);
           absorb "upd" UA~(zA) A~(zA) dA~(zA) UB~(zB) B~(zB) dB~(zB)
  stage 2  squeeze zY (n_T + n_out), zX (n_T + n_in), z2 (n_T + n_r), z4 (n_T + n_r)
  stage 3  six group sumchecks at given points, branch k = 0..5 (fork "fork"):
           {X^T G} = dA at zA, {H^T dY} = dB at zB, {X W, H B} = Y at zY,
           {dY W^T, G A^T} = dX at zX, {X A} = C2 at z2, {dY B^T} = C4 at z4;
           then absorb "join" with the six final states
  stage 4  seven claim reductions on X, W, A, B, dY, H, G, branch j (fork
           "rfork"): absorb "rclaims" v_1..v_K; squeeze rho_1..rho_K; rounds
           over the rows ("round", "r"); absorb "rfinal" t_1(r)..t_K(r);
           squeeze sigma_1..sigma_K; rounds over the columns; absorb "final"
           M~(r, s); then absorb "join" with the seven final states
Proof bytes: the six stage-1 values, the six group proofs (zkmat layout),
then per reduction the row rounds, t_k(r), the column rounds and M~(r, s).
"""
import struct
from typing import Dict, List, Sequence, Tuple

import numpy as np

from .field import P, enc, dec
from .mle import num_vars, eq_basis, eq_table, matrix_mle, partial_eval_rows, partial_eval_cols
from .transcript import Transcript, sha256
from .zkmat import (FalseStatement, Reject, ProofParts, prove_group_at, verify_group_at, round_poly, fold,
                    interpolate_quadratic, proof_len)

DOMAIN = b"VeriLoRA-chain-v1"
TENSORS = ("X", "W", "A", "B", "dY", "H", "G")


def chain_transcript(seed: int, dims, F: int, eta: int) -> Transcript:
    T, d_in, d_out, r = dims
    return Transcript.from_state(sha256(DOMAIN + struct.pack("<QIIIIII", seed, T, d_in, d_out, r, F, eta)))


def _squeeze(tr: Transcript, label: bytes, n: int) -> List[int]:
    return [tr.squeeze(label) for _ in range(n)]


def _nv(dims):
    T, d_in, d_out, r = dims
    return num_vars(T), num_vars(d_in), num_vars(d_out), num_vars(r)


def group_specs(w) -> List[Tuple[str, List[Tuple[str, str, bool, bool]], str]]:
    """The six groups of stage 3: (point name, [(left, right, transL, transR)], C)."""
    return [("zA", [("X", "G", True, False)], "dA"),
            ("zB", [("H", "dY", True, False)], "dB"),
            ("zY", [("X", "W", False, False), ("H", "B", False, False)], "Y"),
            ("zX", [("dY", "W", False, True), ("G", "A", False, True)], "dX"),
            ("z2", [("X", "A", False, False)], "C2"),
            ("z4", [("dY", "B", False, True)], "C4")]


def _op(M: np.ndarray, t: bool) -> np.ndarray:
    return M.T if t else M


def stage_points(tr: Transcript, dims):
    """Stage 1 and 2 points, squeezed in protocol order (stage 1 first)."""
    nT, nin, nout, nr = _nv(dims)
    pts = {"zA": _squeeze(tr, b"zA", nin + nr), "zB": _squeeze(tr, b"zB", nr + nout)}
    return pts


def stage2_points(tr: Transcript, dims):
    nT, nin, nout, nr = _nv(dims)
    return {"zY": _squeeze(tr, b"zY", nT + nout), "zX": _squeeze(tr, b"zX", nT + nin),
            "z2": _squeeze(tr, b"z2", nT + nr), "z4": _squeeze(tr, b"z4", nT + nr)}


def split_point(z, n_rows):
    return list(z[:n_rows]), list(z[n_rows:])


def collect_claims(pts, nv, details, upd) -> Dict[str, List[Tuple[list, list, int]]]:
    """The point-value claims the earlier stages leave on each tensor, in the
    order the reductions take them: (row point, column point, value) on the
    stored matrix.  An operand used transposed, op(M) = M^T, leaves
    (M^T)~(x, y) = M~(y, x).

    details[k] is group k's sumcheck details (u, v, r per product, finals);
    upd holds the stage-1 values."""
    nT, nin, nout, nr = nv
    zA, zB = split_point(pts["zA"], nin), split_point(pts["zB"], nr)
    zY, zX = split_point(pts["zY"], nT), split_point(pts["zX"], nT)
    z2, z4 = split_point(pts["z2"], nT), split_point(pts["z4"], nT)
    d = details
    rP5, (aP5, bP5) = d[0]["r"][0], d[0]["finals"][0]
    rP6, (aP6, bP6) = d[1]["r"][0], d[1]["finals"][0]
    rP1, (aP1, bP1) = d[2]["r"][0], d[2]["finals"][0]
    rP3, (aP3, bP3) = d[2]["r"][1], d[2]["finals"][1]
    rP7, (aP7, bP7) = d[3]["r"][0], d[3]["finals"][0]
    rP8, (aP8, bP8) = d[3]["r"][1], d[3]["finals"][1]
    rP2, (aP2, bP2) = d[4]["r"][0], d[4]["finals"][0]
    rP4, (aP4, bP4) = d[5]["r"][0], d[5]["finals"][0]
    return {
        "X": [(zY[0], rP1, aP1), (z2[0], rP2, aP2), (rP5, zA[0], aP5)],
        "W": [(rP1, zY[1], bP1), (zX[1], rP7, bP7)],
        "A": [(zA[0], zA[1], upd["A"]), (rP2, z2[1], bP2), (zX[1], rP8, bP8)],
        "B": [(zB[0], zB[1], upd["B"]), (rP3, zY[1], bP3), (z4[1], rP4, bP4)],
        "dY": [(z4[0], rP4, aP4), (rP6, zB[1], bP6), (zX[0], rP7, aP7)],
        "H": [(zY[0], rP3, aP3), (rP6, zB[0], aP6)],
        "G": [(rP5, zA[1], bP5), (zX[0], rP8, aP8)],
    }


# ------------------------------------------------------------ reduction ----
def reduce_prove(tr: Transcript, M: np.ndarray, claims) -> Tuple[bytes, dict]:
    """Reduce the claims M~(x_k, y_k) = v_k to one claim M~(r, s) (module
    docstring); tr is the reduction's own branch and is updated."""
    K = len(claims)
    tr.absorb(b"rclaims", b"".join(enc(v) for _, _, v in claims))
    rho = _squeeze(tr, b"rho", K)
    e = [eq_table(x) for x, _, _ in claims]
    t = [partial_eval_cols(M, y) for _, y, _ in claims]
    out = b""
    r = []
    while len(e[0]) > 1:
        g = [0, 0, 0]
        for k in range(K):
            gk = round_poly(e[k], t[k])
            for j in range(3):
                g[j] += rho[k] * gk[j]
        g = [x % P for x in g]
        msg = enc(g[0]) + enc(g[1]) + enc(g[2])
        tr.absorb(b"round", msg)
        out += msg
        ri = tr.squeeze(b"r")
        r.append(ri)
        e = [fold(x, ri) for x in e]
        t = [fold(x, ri) for x in t]
    tfin = [x[0] for x in t]
    msg = b"".join(enc(x) for x in tfin)
    tr.absorb(b"rfinal", msg)
    out += msg
    sigma = _squeeze(tr, b"sigma", K)
    a = partial_eval_rows(M, r)
    ey = [eq_table(y) for _, y, _ in claims]
    b = [sum(sigma[k] * ey[k][j] for k in range(K)) % P for j in range(len(a))]
    s = []
    while len(a) > 1:
        g = round_poly(a, b)
        msg = enc(g[0]) + enc(g[1]) + enc(g[2])
        tr.absorb(b"round", msg)
        out += msg
        si = tr.squeeze(b"r")
        s.append(si)
        a, b = fold(a, si), fold(b, si)
    tr.absorb(b"final", enc(a[0]))
    out += enc(a[0])
    return out, dict(rho=rho, sigma=sigma, r=r, s=s, t=tfin, value=a[0])


def reduce_len(shape, K: int) -> int:
    return 32 * (3 * num_vars(shape[0]) + K + 3 * num_vars(shape[1]) + 1)


def reduce_verify(tr: Transcript, shape, claims, data: bytes) -> dict:
    """Verifier of one reduction; returns the reduced claim (r, s, value)."""
    if len(data) != reduce_len(shape, len(claims)):
        raise Reject("length")
    try:
        el = [dec(data[i:i + 32]) for i in range(0, len(data), 32)]
    except ValueError:
        raise Reject("encoding")
    K = len(claims)
    nR, nC = num_vars(shape[0]), num_vars(shape[1])
    tr.absorb(b"rclaims", b"".join(enc(v) for _, _, v in claims))
    rho = _squeeze(tr, b"rho", K)
    claim = sum(rho[k] * claims[k][2] for k in range(K)) % P
    pos, r = 0, []
    for i in range(nR):
        g0, g1, g2 = el[pos:pos + 3]
        pos += 3
        if (g0 + g1) % P != claim:
            raise Reject("reduction row round", i + 1)
        tr.absorb(b"round", enc(g0) + enc(g1) + enc(g2))
        ri = tr.squeeze(b"r")
        r.append(ri)
        claim = interpolate_quadratic(g0, g1, g2, ri)
    tfin = el[pos:pos + K]
    pos += K
    if sum(rho[k] * eq_basis(claims[k][0], r) * tfin[k] for k in range(K)) % P != claim:
        raise Reject("reduction row final")
    tr.absorb(b"rfinal", b"".join(enc(x) for x in tfin))
    sigma = _squeeze(tr, b"sigma", K)
    claim = sum(sigma[k] * tfin[k] for k in range(K)) % P
    s = []
    for i in range(nC):
        g0, g1, g2 = el[pos:pos + 3]
        pos += 3
        if (g0 + g1) % P != claim:
            raise Reject("reduction column round", nR + i + 1)
        tr.absorb(b"round", enc(g0) + enc(g1) + enc(g2))
        si = tr.squeeze(b"r")
        s.append(si)
        claim = interpolate_quadratic(g0, g1, g2, si)
    value = el[pos]
    if value * sum(sigma[k] * eq_basis(claims[k][1], s) for k in range(K)) % P != claim:
        raise Reject("reduction column final")
    tr.absorb(b"final", enc(value))
    return dict(r=r, s=s, value=value)


# ---------------------------------------------------------------- chain ----
def _tensors(w) -> Dict[str, np.ndarray]:
    return {k: getattr(w, k) for k in ("X", "W", "A", "B", "dY", "H", "G", "Y", "C2", "C4", "dA", "dB", "dX",
                                       "UA", "UB")}


def chain_prove(w, seed: int):
    """Prove one layer's step (w: workloads.LayerWitness).  Returns (proof
    bytes, final transcript state, details).  Raises FalseStatement if the
    update relation or any product group does not hold."""
    dims = w.dims
    nv = _nv(dims)
    nT, nin, nout, nr = nv
    M = _tensors(w)
    tr = chain_transcript(seed, dims, w.F, w.eta)
    # stage 1: the update relation at random points
    pts = stage_points(tr, dims)
    zA, zB = split_point(pts["zA"], nin), split_point(pts["zB"], nr)
    upd = {"UA": matrix_mle(M["UA"], *zA), "A": matrix_mle(M["A"], *zA), "dA": matrix_mle(M["dA"], *zA),
           "UB": matrix_mle(M["UB"], *zB), "B": matrix_mle(M["B"], *zB), "dB": matrix_mle(M["dB"], *zB)}
    for U, X0, D in (("UA", "A", "dA"), ("UB", "B", "dB")):
        if upd[U] != ((1 << w.F) * upd[X0] - w.eta * upd[D]) % P:
            raise FalseStatement(f"{U} differs from 2^F {X0} - eta {D}")
    out = b"".join(enc(upd[k]) for k in ("UA", "A", "dA", "UB", "B", "dB"))
    tr.absorb(b"upd", out)
    # stage 2: points of the outputs and of the cut points
    pts.update(stage2_points(tr, dims))
    # stage 3: the group sumchecks at those points, one branch each
    details, states = [], []
    rows_of = {"zA": nin, "zB": nr, "zY": nT, "zX": nT, "z2": nT, "z4": nT}
    for k, (pname, prods, cname) in enumerate(group_specs(w)):
        u, v = split_point(pts[pname], rows_of[pname])
        br = tr.fork(b"fork", k)
        pr = [(_op(M[a], ta), _op(M[b], tb)) for a, b, ta, tb in prods]
        proof, det = prove_group_at(pr, M[cname], br, u, v)
        out += proof
        details.append(det)
        states.append(br.state)
    tr.absorb(b"join", b"".join(states))
    # stage 4: one claim per tensor
    claims = collect_claims(pts, nv, details, upd)
    reduced, states = {}, []
    for j, name in enumerate(TENSORS):
        br = tr.fork(b"rfork", j)
        proof, det = reduce_prove(br, M[name], claims[name])
        out += proof
        reduced[name] = det
        states.append(br.state)
    tr.absorb(b"join", b"".join(states))
    return out, tr.state, dict(points=pts, upd=upd, groups=details, claims=claims, reduced=reduced)


def chain_proof_len(dims) -> int:
    nv = _nv(dims)
    T, d_in, d_out, r = dims
    shapes_of = {"dA": [(d_in, T, r)], "dB": [(r, T, d_out)], "Y": [(T, d_in, d_out), (T, r, d_out)],
                 "dX": [(T, d_out, d_in), (T, r, d_in)], "C2": [(T, d_in, r)], "C4": [(T, d_out, r)]}
    n = 6 * 32 + sum(proof_len(shapes_of[c]) for _, _, c in group_specs(None))
    mshape = {"X": (T, d_in), "W": (d_in, d_out), "A": (d_in, r), "B": (r, d_out), "dY": (T, d_out),
              "H": (T, r), "G": (T, r)}
    K = {"X": 3, "W": 2, "A": 3, "B": 3, "dY": 3, "H": 2, "G": 2}
    return n + sum(reduce_len(mshape[t], K[t]) for t in TENSORS)


def chain_verify(proof: bytes, dims, seed: int, F: int, eta: int, witness=None) -> dict:
    """Check a chain proof.  Returns the claims left at the end: one per
    tensor of TENSORS (point, value) and the open claims on UA, UB, Y, dX, C2
    and C4.  With a witness (a LayerWitness) every one of them is also
    checked by direct evaluation of eq. (MLE), standing in for the openings
    of committed tensors (out of scope)."""
    T, d_in, d_out, r = dims
    nv = _nv(dims)
    nT, nin, nout, nr = nv
    if len(proof) != chain_proof_len(dims):
        raise Reject("length")
    tr = chain_transcript(seed, dims, F, eta)
    pts = stage_points(tr, dims)
    try:
        vals = [dec(proof[32 * i:32 * i + 32]) for i in range(6)]
    except ValueError:
        raise Reject("encoding")
    upd = dict(zip(("UA", "A", "dA", "UB", "B", "dB"), vals))
    for U, X0, D in (("UA", "A", "dA"), ("UB", "B", "dB")):
        if upd[U] != ((1 << F) * upd[X0] - eta * upd[D]) % P:
            raise Reject("update relation")
    tr.absorb(b"upd", proof[:6 * 32])
    pos = 6 * 32
    pts.update(stage2_points(tr, dims))
    shapes_of = {"dA": [(d_in, T, r)], "dB": [(r, T, d_out)], "Y": [(T, d_in, d_out), (T, r, d_out)],
                 "dX": [(T, d_out, d_in), (T, r, d_in)], "C2": [(T, d_in, r)], "C4": [(T, d_out, r)]}
    rows_of = {"zA": nin, "zB": nr, "zY": nT, "zX": nT, "z2": nT, "z4": nT}
    details, states, opened = [], [], {}
    for k, (pname, _, cname) in enumerate(group_specs(None)):
        u, v = split_point(pts[pname], rows_of[pname])
        n = proof_len(shapes_of[cname])
        br = tr.fork(b"fork", k)
        res = verify_group_at(proof[pos:pos + n], shapes_of[cname], br, u, v)
        pos += n
        res["finals"] = list(res["finals"])
        details.append(res)
        states.append(br.state)
        opened[cname] = (u, v, res["c"])
    if opened["dA"][2] != upd["dA"] or opened["dB"][2] != upd["dB"]:
        raise Reject("update claim differs from its sumcheck's claim")
    tr.absorb(b"join", b"".join(states))
    claims = collect_claims(pts, nv, details, upd)
    mshape = {"X": (T, d_in), "W": (d_in, d_out), "A": (d_in, r), "B": (r, d_out), "dY": (T, d_out),
              "H": (T, r), "G": (T, r)}
    reduced, states = {}, []
    for j, name in enumerate(TENSORS):
        n = reduce_len(mshape[name], len(claims[name]))
        br = tr.fork(b"rfork", j)
        reduced[name] = reduce_verify(br, mshape[name], claims[name], proof[pos:pos + n])
        pos += n
        states.append(br.state)
    tr.absorb(b"join", b"".join(states))
    zA, zB = split_point(pts["zA"], nin), split_point(pts["zB"], nr)
    open_claims = {"UA": (zA[0], zA[1], upd["UA"]), "UB": (zB[0], zB[1], upd["UB"]),
                   "Y": opened["Y"], "dX": opened["dX"], "C2": opened["C2"], "C4": opened["C4"]}
    if witness is not None:
        Mw = _tensors(witness)
        for name, red in reduced.items():
            if matrix_mle(Mw[name], red["r"], red["s"]) != red["value"]:
                raise Reject(f"witness: {name}")
        for name, (x, y, v) in open_claims.items():
            if matrix_mle(Mw[name], x, y) != v:
                raise Reject(f"witness: {name}")
    return dict(reduced=reduced, open=open_claims, state=tr.state, points=pts)
