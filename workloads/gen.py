"""Seeded synthetic inputs shaped like the paper's LoRA fine-tuning matmuls.

The paper proves every matrix product of a LoRA step (forward, backward and
the LoRA update) with its matmul sumcheck (Sections III-IV).  It trains on real
LLaMA/OPT weights and C4 text, neither of which is used here: these generators
draw fixed-point int16 tensors with the shapes of a 7B-class (hidden 4096,
FFN 11008) and a 13B-class (hidden 5120, FFN 13824) decoder layer instead.

Conventions (all integers, nothing here touches a field):
  * Gaussian tensors are quantised as clip(rint(N(0, sigma^2) * 2^12)) to int16;
    sigma = 0.02 for weights (W, LoRA A, LoRA B) and 1 for activations and dY.
  * LoRA layer:  Y = X W + (X A) B,  X: T x d_in, W: d_in x d_out,
    A: d_in x r, B: r x d_out.  Chained operands are re-quantised with
    ``requant`` (round half up at scale 2^12, saturating to int16).
  * Backward and update:  G = requant(dY B^T), dA = X^T G, dB = H^T dY,
    dX = dY W^T + G A^T (a two-product sum group), H = requant(X A).
  * The witness C of a group is the exact integer sum of its products.

Tensors are drawn with ``numpy.random.default_rng(seed)`` in the order each
constructor lists, so a (config, seed) pair always yields the same bytes.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np

SCALE_BITS = 12
I16_MIN, I16_MAX = -(1 << 15), (1 << 15) - 1


# --------------------------------------------------------------------------
# data model
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Product:
    """One product op(A) @ op(B); op is the identity or a transposed view.

    ``A`` and ``B`` are the stored (row-major, C-contiguous) tensors.  The
    mathematical left factor is ``A.T`` when ``transA`` is set, likewise for B.
    """
    name: str
    A: np.ndarray
    B: np.ndarray
    transA: bool = False
    transB: bool = False

    def opA(self) -> np.ndarray:
        return self.A.T if self.transA else self.A

    def opB(self) -> np.ndarray:
        return self.B.T if self.transB else self.B

    @property
    def dims(self):
        a, b = self.opA(), self.opB()
        assert a.shape[1] == b.shape[0], (self.name, a.shape, b.shape)
        return (int(a.shape[0]), int(a.shape[1]), int(b.shape[1]))


@dataclasses.dataclass
class Group:
    """Products that share the output C (C = sum of the products)."""
    name: str
    products: List[Product]
    C: np.ndarray
    group_id: int = 0

    @property
    def shapes(self):
        return [p.dims for p in self.products]


@dataclasses.dataclass
class Workload:
    name: str
    seed: int
    groups: List[Group]

    def n_products(self) -> int:
        return sum(len(g.products) for g in self.groups)


# --------------------------------------------------------------------------
# integer helpers (witness generation only)
# --------------------------------------------------------------------------
def quantize_gaussian(rng: np.random.Generator, shape, sigma: float) -> np.ndarray:
    x = rng.standard_normal(shape) * (sigma * (1 << SCALE_BITS))
    return np.clip(np.rint(x), I16_MIN, I16_MAX).astype(np.int16)


def requant(z: np.ndarray) -> np.ndarray:
    """Round-half-up rescale by 2^12 with int16 saturation (chained operands)."""
    z = np.asarray(z, dtype=np.int64)
    q = (z + (1 << (SCALE_BITS - 1))) >> SCALE_BITS
    return np.clip(q, I16_MIN, I16_MAX).astype(np.int16)


def exact_matmul(a: np.ndarray, b: np.ndarray, device: Optional[str] = None) -> np.ndarray:
    """Exact integer product as int64.

    Large products go through float64 GEMM, which is exact here: every product
    of two entries and every partial sum is an integer of magnitude below 2^53
    (checked from the operand bounds), so no rounding can occur in any order.
    ``device="cuda"`` runs that float64 GEMM with torch on the GPU (witness
    generation for benchmarks); small products use int64 matmul on the host.
    """
    a = np.asarray(a)
    b = np.asarray(b)
    k = a.shape[1]
    amax = int(np.abs(a.astype(np.int64)).max(initial=0))
    bmax = int(np.abs(b.astype(np.int64)).max(initial=0))
    bound = amax * bmax * max(k, 1)
    if bound >= (1 << 53):
        if bound >= (1 << 62):
            raise ValueError("product would overflow int64")
        return a.astype(np.int64) @ b.astype(np.int64)
    if a.shape[0] * k * b.shape[1] <= (1 << 22):
        return a.astype(np.int64) @ b.astype(np.int64)
    if device is not None and device != "cpu":
        import torch
        ta = torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=torch.float64)
        tb = torch.from_numpy(np.ascontiguousarray(b)).to(device=device, dtype=torch.float64)
        out = (ta @ tb).to(torch.int64).cpu().numpy()
        return out
    return (a.astype(np.float64) @ b.astype(np.float64)).astype(np.int64)


def _group(name, prods, device=None) -> Group:
    C = None
    for p in prods:
        t = exact_matmul(p.opA(), p.opB(), device=device)
        C = t if C is None else C + t
    return Group(name, prods, C)


def _number(groups: List[Group]) -> List[Group]:
    for i, g in enumerate(groups):
        g.group_id = i
    return groups


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------
def config1(seed: int = 1) -> Workload:
    """Single product: A 64x128 and B 128x32, int16 uniform in [-2^15, 2^15)."""
    rng = np.random.default_rng(seed)
    A = rng.integers(I16_MIN, I16_MAX + 1, size=(64, 128), dtype=np.int16)
    B = rng.integers(I16_MIN, I16_MAX + 1, size=(128, 32), dtype=np.int16)
    g = _group("A@B", [Product("A@B", A, B)])
    return Workload("single 64x128x32 int16", seed, _number([g]))


class LoraLayer:
    """Draws one LoRA-adapted linear layer: X, W, A, B (and dY on demand)."""

    def __init__(self, rng, T, d_in, d_out, r, with_dy: bool, X: Optional[np.ndarray] = None):
        self.T, self.d_in, self.d_out, self.r = T, d_in, d_out, r
        self.X = quantize_gaussian(rng, (T, d_in), 1.0) if X is None else X
        self.W = quantize_gaussian(rng, (d_in, d_out), 0.02)
        self.A = quantize_gaussian(rng, (d_in, r), 0.02)
        self.B = quantize_gaussian(rng, (r, d_out), 0.02)
        self.dY = quantize_gaussian(rng, (T, d_out), 1.0) if with_dy else None
        self._H = None
        self._G = None

    @property
    def H(self):
        if self._H is None:
            self._H = requant(exact_matmul(self.X, self.A))
        return self._H

    @property
    def G(self):
        if self._G is None:
            self._G = requant(exact_matmul(self.dY, self.B.T))
        return self._G


def lora_forward(L: LoraLayer, tag: str = "", device=None) -> List[Group]:
    """P1 X.W, P2 X.A, P3 H.B."""
    return [
        _group(f"{tag}P1 X.W", [Product(f"{tag}P1 X.W", L.X, L.W)], device),
        _group(f"{tag}P2 X.A", [Product(f"{tag}P2 X.A", L.X, L.A)], device),
        _group(f"{tag}P3 H.B", [Product(f"{tag}P3 H.B", L.H, L.B)], device),
    ]


def lora_backward_update(L: LoraLayer, tag: str = "", device=None) -> List[Group]:
    """P4 G=dY.B^T, P5 dA=X^T.G, P6 dB=H^T.dY, dX = P7 dY.W^T + P8 G.A^T."""
    return [
        _group(f"{tag}P4 dY.B^T", [Product(f"{tag}P4 dY.B^T", L.dY, L.B, transB=True)], device),
        _group(f"{tag}P5 X^T.G", [Product(f"{tag}P5 X^T.G", L.X, L.G, transA=True)], device),
        _group(f"{tag}P6 H^T.dY", [Product(f"{tag}P6 H^T.dY", L.H, L.dY, transA=True)], device),
        _group(f"{tag}dX", [Product(f"{tag}P7 dY.W^T", L.dY, L.W, transB=True),
                            Product(f"{tag}P8 G.A^T", L.G, L.A, transB=True)], device),
    ]


def config2(seed: int = 2, T: int = 512, device=None) -> Workload:
    """LoRA forward of a 4096x4096 layer, rank 16, T tokens: 3 products."""
    rng = np.random.default_rng(seed)
    L = LoraLayer(rng, T, 4096, 4096, 16, with_dy=False)
    return Workload(f"lora fwd T={T} 4096x4096 r16", seed, _number(lora_forward(L, device=device)))


def config3(seed: int = 3, T: int = 512, device=None) -> Workload:
    """Backward + update of the 4096x4096 layer (P4..P8) and the full FFN-up
    layer 4096->11008 (P1..P8), rank 16, T tokens."""
    rng = np.random.default_rng(seed)
    L1 = LoraLayer(rng, T, 4096, 4096, 16, with_dy=True)
    L2 = LoraLayer(rng, T, 4096, 11008, 16, with_dy=True)
    groups = lora_backward_update(L1, "attn:", device) + lora_forward(L2, "up:", device) \
        + lora_backward_update(L2, "up:", device)
    return Workload(f"lora bwd+upd T={T} 4096x4096 + ffn-up 4096x11008 r16", seed, _number(groups))


BLOCK_7B = dict(hidden=4096, ffn=11008, r=16)


def config4(seed: int = 4, T: int = 2048, hidden: int = 4096, ffn: int = 11008, r: int = 16,
            device=None) -> Workload:
    """One decoder block, LoRA rank r on q, k, v, o, gate, up, down; all
    forward, backward and update products (7 targets x 8 products)."""
    rng = np.random.default_rng(seed)
    x_attn = quantize_gaussian(rng, (T, hidden), 1.0)
    x_o = quantize_gaussian(rng, (T, hidden), 1.0)
    x_mlp = quantize_gaussian(rng, (T, hidden), 1.0)
    x_down = quantize_gaussian(rng, (T, ffn), 1.0)
    targets = [("q", x_attn, hidden, hidden), ("k", x_attn, hidden, hidden),
               ("v", x_attn, hidden, hidden), ("o", x_o, hidden, hidden),
               ("gate", x_mlp, hidden, ffn), ("up", x_mlp, hidden, ffn),
               ("down", x_down, ffn, hidden)]
    groups: List[Group] = []
    for name, X, d_in, d_out in targets:
        L = LoraLayer(rng, T, d_in, d_out, r, with_dy=True, X=X)
        groups += lora_forward(L, f"{name}:", device) + lora_backward_update(L, f"{name}:", device)
    return Workload(f"7B block T={T} h{hidden} ffn{ffn} r{r}", seed, _number(groups))


def block_weights(seed: int = 4, hidden: int = 4096, ffn: int = 11008, only=None):
    """The frozen weights of one 7B-class decoder block, the matrices a
    commitment covers: W_q, W_k, W_v, W_o (hidden x hidden), W_gate, W_up
    (hidden x ffn) and W_down (ffn x hidden), int16 quantised Gaussians with
    sigma 0.02 at scale 2^12 (as the LoRA layers above).  ``only``: a subset
    of the names (each matrix has a generator of its own, seeded by
    (seed, index), so a subset draws the same values)."""
    shapes = [("q", hidden, hidden), ("k", hidden, hidden), ("v", hidden, hidden), ("o", hidden, hidden),
              ("gate", hidden, ffn), ("up", hidden, ffn), ("down", ffn, hidden)]
    out = []
    for k, (name, r, c) in enumerate(shapes):
        if only is not None and name not in only:
            continue
        out.append((name, quantize_gaussian(np.random.default_rng([seed, k]), (r, c), 0.02)))
    return out


# --------------------------------------------------------------------------
# one LoRA layer as a chain of claims (forward, backward and update)
# --------------------------------------------------------------------------
CHAIN_F, CHAIN_ETA = 12, 3   # update U = 2^F A - eta dA (eta at scale 2^-12: about 7e-4)


@dataclasses.dataclass
class LayerWitness:
    """Every tensor of one LoRA layer's training step, as integers.

    Inputs (int16): X (T x d_in), W (d_in x d_out), A (d_in x r), B (r x d_out),
    dY (T x d_out) and the re-quantised intermediates H = requant(X A) and
    G = requant(dY B^T) (T x r).  Exact int64 results: Y = X W + H B,
    C2 = X A, C4 = dY B^T, dA = X^T G, dB = H^T dY, dX = dY W^T + G A^T and the
    pre-rounding updates UA = 2^F A - eta dA, UB = 2^F B - eta dB."""
    X: np.ndarray
    W: np.ndarray
    A: np.ndarray
    B: np.ndarray
    dY: np.ndarray
    H: np.ndarray
    G: np.ndarray
    Y: np.ndarray
    C2: np.ndarray
    C4: np.ndarray
    dA: np.ndarray
    dB: np.ndarray
    dX: np.ndarray
    UA: np.ndarray
    UB: np.ndarray
    F: int = CHAIN_F
    eta: int = CHAIN_ETA

    @property
    def dims(self):
        return (int(self.X.shape[0]), int(self.X.shape[1]), int(self.W.shape[1]), int(self.A.shape[1]))


def layer_witness(L: "LoraLayer", F: int = CHAIN_F, eta: int = CHAIN_ETA, device=None) -> LayerWitness:
    """All tensors of one layer's step from a drawn LoraLayer (with dY)."""
    X, W, A, B, dY, H, G = L.X, L.W, L.A, L.B, L.dY, L.H, L.G
    mm = lambda a, b: exact_matmul(a, b, device=device)  # noqa: E731
    C2 = exact_matmul(X, A)
    C4 = exact_matmul(dY, B.T)
    Y = mm(X, W) + mm(H, B)
    dA = mm(X.T, G)
    dB = mm(H.T, dY)
    dX = mm(dY, W.T) + mm(G, A.T)
    UA = (A.astype(np.int64) << F) - eta * dA
    UB = (B.astype(np.int64) << F) - eta * dB
    return LayerWitness(X, W, A, B, dY, H, G, Y, C2, C4, dA, dB, dX, UA, UB, F, eta)


def chain_layer(seed: int = 3, T: int = 512, d_in: int = 4096, d_out: int = 11008, r: int = 16,
                device=None) -> LayerWitness:
    """The FFN-up layer of the backward-and-update configuration (T = 512,
    4096 -> 11008, rank 16) as one chained step: the same draw order as
    config3's second layer, from a generator of its own seed."""
    rng = np.random.default_rng([seed, 77])
    L = LoraLayer(rng, T, d_in, d_out, r, with_dy=True)
    return layer_witness(L, device=device)


def tiny_layer(seed: int, T: int, d_in: int, d_out: int, r: int) -> LayerWitness:
    """A small layer with the same distributions (chain parity cases)."""
    rng = np.random.default_rng([seed, 78])
    L = LoraLayer(rng, T, d_in, d_out, r, with_dy=True)
    return layer_witness(L)


# --------------------------------------------------------------------------
# serving requests (13B-class shapes)
# --------------------------------------------------------------------------
SERVE_13B = dict(hidden=5120, ffn=13824)
SERVE_TARGETS = ("q", "k", "v", "o", "gate", "up", "down")
SERVE_T = (128, 512, 2048)
SERVE_RANKS = (8, 16, 64)
SERVE_TYPES = ("fwd", "bwd", "upd")


def serve_dims(target: str, hidden: int = 5120, ffn: int = 13824):
    if target in ("q", "k", "v", "o"):
        return hidden, hidden
    if target in ("gate", "up"):
        return hidden, ffn
    return ffn, hidden


def frozen_weight(target: str, seed: int = 5, hidden: int = 5120, ffn: int = 13824) -> np.ndarray:
    """The frozen W of one target; shared by every request on that target."""
    d_in, d_out = serve_dims(target, hidden, ffn)
    rng = np.random.default_rng([seed, SERVE_TARGETS.index(target)])
    return quantize_gaussian(rng, (d_in, d_out), 0.02)


def serving_request(req_id: int, target: str, T: int, r: int, kind: str, W: np.ndarray,
                    seed: int = 5, device=None) -> Workload:
    """One proof request: fwd -> P1..P3, bwd -> P4 + dX group, upd -> P5, P6."""
    d_in, d_out = W.shape
    rng = np.random.default_rng([seed, 1000 + req_id])
    X = quantize_gaussian(rng, (T, d_in), 1.0)
    L = LoraLayer.__new__(LoraLayer)
    L.T, L.d_in, L.d_out, L.r = T, d_in, d_out, r
    L.X, L.W = X, W
    L.A = quantize_gaussian(rng, (d_in, r), 0.02)
    L.B = quantize_gaussian(rng, (r, d_out), 0.02)
    L.dY = quantize_gaussian(rng, (T, d_out), 1.0) if kind != "fwd" else None
    L._H = None
    L._G = None
    tag = f"req{req_id}:{target}:"
    if kind == "fwd":
        groups = lora_forward(L, tag, device)
    else:
        bu = lora_backward_update(L, tag, device)
        groups = [bu[0], bu[3]] if kind == "bwd" else [bu[1], bu[2]]
    return Workload(f"request {req_id} {kind} {target} T={T} r={r}", seed, _number(groups))


def serving_stream(n: int, rate_per_s: float, seed: int = 5):
    """Poisson arrival times and request types: list of (t_arrive, target, T, r, kind)."""
    rng = np.random.default_rng([seed, 7])
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    t = np.cumsum(gaps)
    out = []
    for i in range(n):
        out.append((float(t[i]), SERVE_TARGETS[rng.integers(len(SERVE_TARGETS))],
                    SERVE_T[rng.integers(len(SERVE_T))], SERVE_RANKS[rng.integers(len(SERVE_RANKS))],
                    SERVE_TYPES[rng.integers(len(SERVE_TYPES))]))
    return out


def serving_sample(n: int = 12):
    """A fixed request mix for parity checks at 13B-class shapes: list of
    (target, T, rank, kind) covering every target, every T, every rank and
    every request type at least once (n >= 7).  Request k takes target k mod 7,
    T index k mod 3, rank index floor(k / 3) mod 3 and type index
    (k + floor(k / 3)) mod 3, so the pairs (T, rank) and (T, type) vary too."""
    if n < 7:
        raise ValueError("the sample needs at least 7 requests to cover every target")
    out = []
    for k in range(n):
        out.append((SERVE_TARGETS[k % 7], SERVE_T[k % 3], SERVE_RANKS[(k // 3) % 3],
                    SERVE_TYPES[(k + k // 3) % 3]))
    return out


def serving_sample_workload(k: int, spec, weights=None, seed: int = 5, device=None) -> Workload:
    """Request k of ``serving_sample`` as a Workload whose seed is the seed its
    proof is made with (5000 + k); ``weights`` caches the frozen W per target."""
    target, T, r, kind = spec
    if weights is None:
        weights = {}
    if target not in weights:
        weights[target] = frozen_weight(target, seed=seed)
    w = serving_request(k, target, T, r, kind, weights[target], seed=seed, device=device)
    w.seed = 5000 + k
    return w


# --------------------------------------------------------------------------
# small random groups for parity tests
# --------------------------------------------------------------------------
_DTYPE_RANGE = {np.int16: (I16_MIN, I16_MAX), np.int32: (-(1 << 31), (1 << 31) - 1),
                np.int64: (-(1 << 62), (1 << 62) - 1)}


def tiny_random_group(seed: int, dims_list, dtype=np.int16, trans=(False, False),
                      value_bits: Optional[int] = None, name: str = "rand") -> Group:
    """A group of products with the given (D0, D1, D2) dims (shared D0, D2).

    Entries are uniform over the dtype (or over +-2^value_bits if given).  The
    stored tensors are transposed when the matching flag is set, so that the
    product is formed through a transposed view.
    """
    rng = np.random.default_rng(seed)
    lo, hi = _DTYPE_RANGE[dtype]
    if value_bits is not None:
        lo, hi = -(1 << value_bits), (1 << value_bits) - 1
    prods = []
    for k, (d0, d1, d2) in enumerate(dims_list):
        a = rng.integers(lo, hi + 1, size=(d0, d1), dtype=np.int64).astype(dtype)
        b = rng.integers(lo, hi + 1, size=(d1, d2), dtype=np.int64).astype(dtype)
        A = np.ascontiguousarray(a.T) if trans[0] else a
        B = np.ascontiguousarray(b.T) if trans[1] else b
        prods.append(Product(f"{name}{k}", A, B, transA=trans[0], transB=trans[1]))
    g = _group(name, prods)
    return g


CONFIG_NAMES = ("cfg1", "cfg2", "cfg3", "cfg4")


def make_config(name: str, **kw) -> Workload:
    fn: Callable[..., Workload] = {"cfg1": config1, "cfg2": config2, "cfg3": config3,
                                   "cfg4": config4}[name]
    return fn(**kw)


# --------------------------------------------------------------------------
# per-head (batched) products: multi-head attention
# --------------------------------------------------------------------------
@dataclasses.dataclass
class HeadView:
    """H matrices of one shape inside one stored, C-contiguous array: head k
    is the rows x cols matrix at element offset k * head_stride, row-major with
    leading dimension ld (in elements)."""
    base: np.ndarray
    H: int
    rows: int
    cols: int
    head_stride: int
    ld: int

    def heads(self) -> np.ndarray:
        flat = self.base.reshape(-1)
        es = flat.itemsize
        need = (self.H - 1) * self.head_stride + (self.rows - 1) * self.ld + self.cols
        assert need <= flat.size and self.cols <= self.ld
        return np.lib.stride_tricks.as_strided(flat, shape=(self.H, self.rows, self.cols),
                                               strides=(self.head_stride * es, self.ld * es, es),
                                               writeable=False)


@dataclasses.dataclass
class HeadBatch:
    """C_k = op(A_k) op(B_k) for every head k (op: identity or transpose of
    the stored head matrix)."""
    name: str
    A: HeadView
    B: HeadView
    C: HeadView
    transA: bool = False
    transB: bool = False
    group_id: int = 0

    def opA_heads(self) -> List[np.ndarray]:
        return [m.T if self.transA else m for m in self.A.heads()]

    def opB_heads(self) -> List[np.ndarray]:
        return [m.T if self.transB else m for m in self.B.heads()]

    def C_heads(self) -> List[np.ndarray]:
        return list(self.C.heads())

    @property
    def dims(self):
        a, b = self.opA_heads()[0], self.opB_heads()[0]
        assert a.shape[1] == b.shape[0]
        return (self.A.H, int(a.shape[0]), int(a.shape[1]), int(b.shape[1]))


def cols_heads(M: np.ndarray, H: int) -> HeadView:
    """Heads side by side in the columns of a T x (H * dh) matrix."""
    T, W = M.shape
    dh = W // H
    return HeadView(M, H, T, dh, dh, W)


def stacked_heads(M: np.ndarray) -> HeadView:
    """Heads stacked in the leading index of an H x rows x cols array."""
    H, R, Cc = M.shape
    return HeadView(M, H, R, Cc, R * Cc, Cc)


def _batched_witness(A: HeadView, B: HeadView, transA: bool, transB: bool, out_shape, out_view,
                     device=None) -> HeadView:
    C = np.zeros(out_shape, dtype=np.int64)
    view = out_view(C)
    ah, bh = A.heads(), B.heads()
    for k in range(A.H):
        a = ah[k].T if transA else ah[k]
        b = bh[k].T if transB else bh[k]
        res = exact_matmul(np.ascontiguousarray(a), np.ascontiguousarray(b), device=device)
        flat = C.reshape(-1)
        for i in range(res.shape[0]):
            o = k * view.head_stride + i * view.ld
            flat[o:o + res.shape[1]] = res[i]
    return view


_EXP_TAB = None


def int_softmax(S: np.ndarray, dh: int) -> np.ndarray:
    """Row softmax of S / (2^24 sqrt(dh)) quantised at scale 2^12, in integer
    arithmetic so that every machine draws the same bytes: the gap to the
    row maximum is cut to k = floor(256 * gap) (at most 4095), exp(-k / 256)
    comes from a table of round(2^20 exp(-k / 256)), and each row is
    normalised by integer division with rounding."""
    global _EXP_TAB
    import math
    if _EXP_TAB is None:
        _EXP_TAB = np.array([int(round(math.exp(-k / 256.0) * (1 << 20))) for k in range(4096)], dtype=np.int64)
    q = int(round((1 << 24) * math.sqrt(dh) / 256.0))
    S = np.asarray(S, dtype=np.int64)
    k = np.minimum((S.max(axis=1, keepdims=True) - S) // q, 4095)
    e = _EXP_TAB[k]
    tot = e.sum(axis=1, keepdims=True)
    return ((e * (1 << SCALE_BITS) + tot // 2) // tot).astype(np.int16)


def attention_layer(seed: int = 6, T: int = 2048, H: int = 32, dh: int = 128, device=None) -> List[HeadBatch]:
    """The per-head products of one attention layer's forward and backward
    pass (7B-class: 32 heads of dimension 128): S = Q K^T, O = P V,
    dP = dO V^T, dV = P^T dO, dQ = dS K, dK = dS^T Q for every head.

    Q, K, V, dO are T x (H dh) int16 activations (sigma = 1 at scale 2^12).
    P is the row softmax of S / (2^24 sqrt(dh)) quantised at scale 2^12
    (entries 0..4096, ``int_softmax``); dS is drawn like an activation
    (H x T x T).  Softmax and
    its gradient are not proved here (lookup arguments); P and dS are witness
    inputs.  S and dP are stored H x T x T, O, dV, dQ, dK as T x (H dh)."""
    rng = np.random.default_rng([seed, 91])
    Q = quantize_gaussian(rng, (T, H * dh), 1.0)
    K = quantize_gaussian(rng, (T, H * dh), 1.0)
    V = quantize_gaussian(rng, (T, H * dh), 1.0)
    dO = quantize_gaussian(rng, (T, H * dh), 1.0)
    dS = quantize_gaussian(rng, (H, T, T), 1.0)
    q, k, v, do = cols_heads(Q, H), cols_heads(K, H), cols_heads(V, H), cols_heads(dO, H)
    ds = stacked_heads(dS)
    tt = (H, T, T)
    S = _batched_witness(q, k, False, True, tt, stacked_heads, device)
    P = np.empty(tt, dtype=np.int16)
    for h in range(H):
        P[h] = int_softmax(S.base[h], dh)
    p = stacked_heads(P)
    cols = lambda M: cols_heads(M, H)  # noqa: E731
    O = _batched_witness(p, v, False, False, (T, H * dh), cols, device)
    dP = _batched_witness(do, v, False, True, tt, stacked_heads, device)
    dV = _batched_witness(p, do, True, False, (T, H * dh), cols, device)
    dQ = _batched_witness(ds, k, False, False, (T, H * dh), cols, device)
    dK = _batched_witness(ds, q, True, False, (T, H * dh), cols, device)
    out = [HeadBatch("S=QK^T", q, k, S, False, True), HeadBatch("O=PV", p, v, O, False, False),
           HeadBatch("dP=dOV^T", do, v, dP, False, True), HeadBatch("dV=P^TdO", p, do, dV, True, False),
           HeadBatch("dQ=dSK", ds, k, dQ, False, False), HeadBatch("dK=dS^TQ", ds, q, dK, True, False)]
    for i, b in enumerate(out):
        b.group_id = i
    return out


def tiny_head_batch(seed: int, H: int, d0: int, d1: int, d2: int, transA: bool = False, transB: bool = False,
                    a_cols: bool = False, b_cols: bool = False, c_cols: bool = False,
                    value_bits: Optional[int] = None, name: str = "bmm") -> HeadBatch:
    """H random heads of op(A) d0 x d1 and op(B) d1 x d2 (int16, uniform, or
    within +-2^value_bits).  *_cols: that operand's heads sit side by side in
    the columns of one matrix (as Q, K, V do), else stacked in an
    H x rows x cols array; the stored head matrix is op's transpose when the
    trans flag is set."""
    rng = np.random.default_rng([seed, 92])
    lo, hi = I16_MIN, I16_MAX
    if value_bits is not None:
        lo, hi = -(1 << value_bits), (1 << value_bits) - 1

    def draw(rows, cols, side):
        if side:
            M = rng.integers(lo, hi + 1, size=(rows, H * cols), dtype=np.int64).astype(np.int16)
            return cols_heads(M, H)
        M = rng.integers(lo, hi + 1, size=(H, rows, cols), dtype=np.int64).astype(np.int16)
        return stacked_heads(M)

    A = draw(d1, d0, a_cols) if transA else draw(d0, d1, a_cols)
    B = draw(d2, d1, b_cols) if transB else draw(d1, d2, b_cols)
    if c_cols:
        C = _batched_witness(A, B, transA, transB, (d0, H * d2), lambda M: cols_heads(M, H))
    else:
        C = _batched_witness(A, B, transA, transB, (H, d0, d2), stacked_heads)
    return HeadBatch(name, A, B, C, transA, transB)


# --------------------------------------------------------------------------
# lookup arguments: entries of a tensor (or pairs of tensors) in a table
# --------------------------------------------------------------------------
@dataclasses.dataclass
class LookupCase:
    """Every x_i (with y_i when y is given) is a row of the table
    (t0 + j, tb_j), j < N: a range check when tb is None, an input/output
    check of an element-wise function otherwise."""
    name: str
    x: np.ndarray
    y: Optional[np.ndarray]
    t0: int
    tb: Optional[np.ndarray]
    N: int
    lid: int = 0


_SILU_TAB = None


def silu_table() -> np.ndarray:
    """SiLU at scale 2^12 over the int16 range: round(2^12 s sigmoid(s)) for
    s = x / 2^12, x = -2^15 .. 2^15 - 1 (int32).  Computed with the C
    library's exp, entry by entry, so that every machine builds the same
    table."""
    global _SILU_TAB
    import math
    if _SILU_TAB is None:
        out = np.empty(1 << 16, dtype=np.int32)
        for j in range(1 << 16):
            s = (j + I16_MIN) / float(1 << SCALE_BITS)
            out[j] = int(round(s / (1.0 + math.exp(-s)) * (1 << SCALE_BITS)))
        _SILU_TAB = out
    return _SILU_TAB


def lookup_range(seed: int, D: int, lid: int = 0) -> LookupCase:
    """Range check of D quantised activations (sigma = 1 at scale 2^12) against
    the int16 table -2^15 .. 2^15 - 1 (N = 2^16)."""
    rng = np.random.default_rng([seed, 93])
    x = quantize_gaussian(rng, (D,), 1.0)
    return LookupCase(f"range D={D}", x, None, I16_MIN, None, 1 << 16, lid)


def lookup_silu(seed: int, D: int, lid: int = 0) -> LookupCase:
    """SwiGLU's activation check (input z', output phi(z')) as a two-column
    lookup into the SiLU table over the int16 range (N = 2^16)."""
    rng = np.random.default_rng([seed, 94])
    x = quantize_gaussian(rng, (D,), 1.0)
    tab = silu_table()
    y = tab[x.astype(np.int64) - I16_MIN].astype(np.int32)
    return LookupCase(f"silu D={D}", x, y, I16_MIN, tab, 1 << 16, lid)


def tiny_lookup(seed: int, D: int, N: int, t0: int = 0, two_col: bool = False, lid: int = 0) -> LookupCase:
    """D entries drawn uniformly from a table of N rows starting at t0 (int32;
    the second column, if any, random int32)."""
    rng = np.random.default_rng([seed, 95])
    j = rng.integers(0, N, size=D)
    x = (t0 + j).astype(np.int32)
    tb = rng.integers(-(1 << 30), 1 << 30, size=N).astype(np.int32) if two_col else None
    y = tb[j].astype(np.int32) if two_col else None
    return LookupCase(f"tiny lookup D={D} N={N}", x, y, t0, tb, N, lid)
