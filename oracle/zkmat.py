"""The matmul sumcheck, prover and verifier (oracle; test infrastructure).

Statement (Sec. II-C, eq. (matmul) and eq. (zk-mle-matmul)): for A (D0 x D1),
B (D1 x D2) and a claimed C (D0 x D2), all zero padded to powers of two,
C = A B holds iff for random u, v
    C~(u, v) = sum_{w in {0,1}^{n1}} A~(u, w) B~(w, v).
The prover turns that sum into a sumcheck over w (Sec. II-B.1): one round per
variable of w, each round a univariate polynomial of degree <= 2, then a random
challenge that fixes the variable.

Readings of the paper taken here (the paper is silent or inconsistent):
  * u and v are random challenges and only w is summed (n1 rounds); the text
    counts d0 + d1 + d2 rounds while saying u, v are Boolean, which cannot both
    hold.  The sent claim is c = C~(u, v), the form equivalent to summing
    D1^-1 C~(u,v) - A~B~ to zero.
  * Round i binds the most significant remaining bit of w, so the halves of
    the current table are paired as (t, t + h).
  * A round message is the three values g(0), g(1), g(2).
  * Matrix additions (zkMat covers additions too, Sec. IV-B): a group whose C
    is a sum of k products shares one transcript and one (u, v); the prover
    sends the part claims s_1..s_{k-1} and then runs the k sumchecks in order,
    the last claim being c - sum of the parts.
  * Each group has its own transcript keyed by (seed, group id, shapes).
  * Commitments before challenges (Sec. II-C: the verifier draws its point
    only after the prover has committed to the matrices, Sec. II-A): a
    caller that holds commitments passes a 32-byte digest of them as
    ``bind``, absorbed with label "bind" right after the initial state and
    before u and v.  Without one the challenges depend only on public data
    and on the prover's messages, and nothing ties C to them.

Proof bytes: c || s_1..s_{k-1} || for each product (g0, g1, g2) per round ||
a_final || b_final, each a 32-byte canonical little-endian field element.
"""
import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

from .field import P, lift, enc, dec, inv
from .mle import num_vars, eq_table, matrix_mle, partial_eval_rows, partial_eval_cols, mle_eval
from .transcript import Transcript

INV2 = inv(2)


class FalseStatement(Exception):
    """The claimed C is not the (sum of the) products: no proof exists."""


class Reject(Exception):
    def __init__(self, reason: str, round_index: int = -1):
        super().__init__(f"{reason} (round {round_index})")
        self.reason = reason
        self.round_index = round_index


@dataclasses.dataclass
class ProofParts:
    c: int
    parts: List[int]
    rounds: List[List[Tuple[int, int, int]]]
    finals: List[Tuple[int, int]]

    def to_bytes(self) -> bytes:
        out = enc(self.c) + b"".join(enc(s) for s in self.parts)
        for rs, (af, bf) in zip(self.rounds, self.finals):
            for g in rs:
                out += enc(g[0]) + enc(g[1]) + enc(g[2])
            out += enc(af) + enc(bf)
        return out

    @staticmethod
    def from_bytes(data: bytes, shapes) -> "ProofParts":
        if len(data) != proof_len(shapes):
            raise Reject("length")
        try:
            el = [dec(data[i:i + 32]) for i in range(0, len(data), 32)]
        except ValueError:
            raise Reject("encoding")
        pos = 0
        c = el[pos]; pos += 1
        parts = el[pos:pos + len(shapes) - 1]; pos += len(shapes) - 1
        rounds, finals = [], []
        for (_, d1, _) in shapes:
            n1 = num_vars(d1)
            rs = []
            for _ in range(n1):
                rs.append((el[pos], el[pos + 1], el[pos + 2])); pos += 3
            rounds.append(rs)
            finals.append((el[pos], el[pos + 1])); pos += 2
        return ProofParts(c, parts, rounds, finals)


def proof_len(shapes) -> int:
    n = 1 + (len(shapes) - 1)
    for (_, d1, _) in shapes:
        n += 3 * num_vars(d1) + 2
    return 32 * n


def group_shapes_ok(shapes) -> None:
    if not shapes:
        raise ValueError("empty group")
    d0, _, d2 = shapes[0]
    for s in shapes:
        if s[0] != d0 or s[2] != d2 or min(s) < 1:
            raise ValueError("products of a group must share D0 and D2")


def challenges_uv(tr: Transcript, shapes):
    d0, _, d2 = shapes[0]
    u = [tr.squeeze(b"u") for _ in range(num_vars(d0))]
    v = [tr.squeeze(b"v") for _ in range(num_vars(d2))]
    return u, v


def claim_value(C: np.ndarray, u, v) -> int:
    """c = C~(u, v) = sum_i eq(u, i) * (sum_j C[i, j] eq(v, j))."""
    t = partial_eval_cols(C, v)
    eu = eq_table(u)
    return sum(eu[i] * t[i] for i in range(len(t))) % P


def round_poly(a: Sequence[int], b: Sequence[int]) -> Tuple[int, int, int]:
    """g(X) = sum_t (a_t + X (a_{t+h} - a_t)) (b_t + X (b_{t+h} - b_t)) at X = 0, 1, 2."""
    h = len(a) // 2
    g0 = sum(a[t] * b[t] for t in range(h)) % P
    g1 = sum(a[t + h] * b[t + h] for t in range(h)) % P
    g2 = sum((2 * a[t + h] - a[t]) * (2 * b[t + h] - b[t]) for t in range(h)) % P
    return g0, g1, g2


def fold(a: Sequence[int], r: int) -> List[int]:
    """Fix the leading variable to r: a'_t = a_t + r (a_{t+h} - a_t)."""
    h = len(a) // 2
    return [(a[t] + r * (a[t + h] - a[t])) % P for t in range(h)]


def interpolate_quadratic(g0: int, g1: int, g2: int, r: int) -> int:
    """The degree-2 polynomial through (0,g0), (1,g1), (2,g2), evaluated at r."""
    l0 = (r - 1) * (r - 2) * INV2
    l1 = -r * (r - 2)
    l2 = r * (r - 1) * INV2
    return (g0 * l0 + g1 * l1 + g2 * l2) % P


def group_transcript(seed: int, group_id: int, shapes, bind: Optional[bytes] = None) -> Transcript:
    """A group's transcript before its challenges: the initial state, then
    the commitments' digest when one is given (Sec. II-C after II-A)."""
    tr = Transcript(seed, group_id, shapes)
    if bind is not None:
        bind = bytes(bind)
        if len(bind) != 32:
            raise ValueError("a bind digest is 32 bytes")
        tr.absorb(b"bind", bind)
    return tr


def prove_group(prods: Sequence[Tuple[np.ndarray, np.ndarray]], C: np.ndarray, seed: int,
                group_id: int, bind: Optional[bytes] = None):
    """Prove C = sum_k A_k B_k.  ``prods`` holds the integer factors as they
    enter the product (transposed views already applied); ``bind`` the
    optional 32-byte digest of the caller's commitments.

    Returns (proof bytes, final transcript state, details dict).
    Raises FalseStatement if the products do not sum to C.
    """
    shapes = [(int(A.shape[0]), int(A.shape[1]), int(B.shape[1])) for A, B in prods]
    group_shapes_ok(shapes)
    for (A, B) in prods:
        assert A.shape[1] == B.shape[0]
    assert C.shape == (shapes[0][0], shapes[0][2])

    tr = group_transcript(seed, group_id, shapes, bind)
    u, v = challenges_uv(tr, shapes)
    proof, details = prove_group_at(prods, C, tr, u, v)
    return proof, tr.state, details


def prove_group_at(prods: Sequence[Tuple[np.ndarray, np.ndarray]], C: np.ndarray, tr: Transcript, u, v):
    """The sumcheck of a group at a given point (u, v), continuing the
    transcript tr (which this updates): the steps of prove_group after the
    challenges.  Used on its own when the point comes from an earlier step
    of a chained proof.  Returns (proof bytes, details)."""
    shapes = [(int(A.shape[0]), int(A.shape[1]), int(B.shape[1])) for A, B in prods]
    group_shapes_ok(shapes)
    c = claim_value(C, u, v)
    tr.absorb(b"claim", enc(c))

    tables = []
    sums = []
    for (A, B) in prods:
        a = partial_eval_rows(A, u)      # a[w] = A~(u, w)
        b = partial_eval_cols(B, v)      # b[w] = B~(w, v)
        tables.append((a, b))
        sums.append(sum(x * y for x, y in zip(a, b)) % P)
    if sum(sums) % P != c:
        raise FalseStatement("sum of A~(u,w) B~(w,v) over w differs from C~(u,v)")

    parts = sums[:-1]
    for s in parts:
        tr.absorb(b"part", enc(s))

    all_rounds, finals, all_r = [], [], []
    for (a, b) in tables:
        rs, rvec = [], []
        while len(a) > 1:
            g = round_poly(a, b)
            tr.absorb(b"round", enc(g[0]) + enc(g[1]) + enc(g[2]))
            r = tr.squeeze(b"r")
            a, b = fold(a, r), fold(b, r)
            rs.append(g)
            rvec.append(r)
        tr.absorb(b"final", enc(a[0]) + enc(b[0]))
        all_rounds.append(rs)
        finals.append((a[0], b[0]))
        all_r.append(rvec)

    pp = ProofParts(c, parts, all_rounds, finals)
    details = dict(u=u, v=v, c=c, sums=sums, r=all_r, finals=finals, rounds=all_rounds)
    return pp.to_bytes(), details


def verify_group(proof: bytes, shapes, seed: int, group_id: int,
                 witness: Optional[Tuple[Sequence[Tuple[np.ndarray, np.ndarray]], np.ndarray]] = None,
                 bind: Optional[bytes] = None):
    """Check a proof; returns the reduced claims, raises Reject.

    Without a witness this checks the sumcheck itself: g(0) + g(1) equals the
    running claim each round, the claim moves to g(r), and the last claim is
    a_final * b_final.  With a witness ((A_k, B_k) list, C) it also checks
    c = C~(u, v), a_final = A~(u, r) and b_final = B~(r, v) by direct
    evaluation, which stands in for commitment openings.  ``bind``: the
    digest the prover bound (the verifier recomputes it from the commitments
    it holds and then checks the reduced claims by openings).
    """
    shapes = [tuple(int(x) for x in s) for s in shapes]
    group_shapes_ok(shapes)
    tr = group_transcript(seed, group_id, shapes, bind)
    u, v = challenges_uv(tr, shapes)
    return verify_group_at(proof, shapes, tr, u, v, witness)


def verify_group_at(proof: bytes, shapes, tr: Transcript, u, v,
                    witness: Optional[Tuple[Sequence[Tuple[np.ndarray, np.ndarray]], np.ndarray]] = None):
    """verify_group at a given point (u, v), continuing the transcript tr
    (which this updates)."""
    shapes = [tuple(int(x) for x in s) for s in shapes]
    group_shapes_ok(shapes)
    pp = ProofParts.from_bytes(proof, shapes)
    tr.absorb(b"claim", enc(pp.c))
    for s in pp.parts:
        tr.absorb(b"part", enc(s))
    claims = list(pp.parts) + [(pp.c - sum(pp.parts)) % P]

    round_no = 0
    all_r = []
    for k, (rs, (af, bf)) in enumerate(zip(pp.rounds, pp.finals)):
        claim = claims[k]
        rvec = []
        for (g0, g1, g2) in rs:
            round_no += 1
            if (g0 + g1) % P != claim:
                raise Reject("round", round_no)
            tr.absorb(b"round", enc(g0) + enc(g1) + enc(g2))
            r = tr.squeeze(b"r")
            claim = interpolate_quadratic(g0, g1, g2, r)
            rvec.append(r)
        if af * bf % P != claim:
            raise Reject("final", round_no)
        tr.absorb(b"final", enc(af) + enc(bf))
        all_r.append(rvec)

    if witness is not None:
        prods, C = witness
        if matrix_mle(C, u, v) != pp.c:
            raise Reject("witness")
        for (A, B), rvec, (af, bf) in zip(prods, all_r, pp.finals):
            if matrix_mle(A, u, rvec) != af or matrix_mle(B, rvec, v) != bf:
                raise Reject("witness")
    return dict(u=u, v=v, c=pp.c, r=all_r, finals=pp.finals, state=tr.state, parts=pp.parts)


def prove_workload_group(group, seed: int, bind: Optional[bytes] = None):
    """Convenience: prove a ``workloads.Group`` (op views applied here)."""
    prods = [(p.opA(), p.opB()) for p in group.products]
    return prove_group(prods, group.C, seed, group.group_id, bind)


def lifted(M: np.ndarray) -> List[List[int]]:
    return [[lift(x) for x in row] for row in M]
