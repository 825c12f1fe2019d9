"""Launch-shape planner: picks vl_tuning per shape signature, cached.

The prover's launch shapes (contraction chunk size, pipeline segments, rows
per lane of the column kernels, the claim's contraction order) change how
the work is cut into GPU tasks, never a byte of the proofs.  The best choice
depends on the shapes of the groups in a call, so the planner keys a cache
by a signature of those shapes (dimensions, dtypes, transposed views, group
structure; not the data), and on a miss times a grid of candidates on the
call's own inputs with the blocking entry point and keeps the fastest.  The
cache lives in memory and, when a path is given, in a JSON file that later
processes load.  Host-side orchestration only: every candidate runs the
library's kernels.
"""
import hashlib
import json
import os
import time
from typing import Dict, List, Optional, Sequence

from . import binding as B

# candidate launch shapes: (lane_macs, segments, cols_rows, claim_order);
# 0 keeps the library default for that knob
DEFAULT_GRID = [(lm, sg, cr, co) for lm in (4096, 8192, 16384) for sg in (1, 2) for cr in (1, 2)
                for co in (0, 1)]
# the library's defaults for those knobs (vl_tuning fields left at 0) in the
# blocking calls the planner times; a persistent call defaults to 4 segments
LIBRARY_DEFAULTS = (8192, 2, 1, 0)


def _defaults(mode: int) -> tuple:
    return (8192, 4, 1, 0) if mode == B.VL_MODE_PERSISTENT else LIBRARY_DEFAULTS


def _resolved(c, mode: int) -> tuple:
    return tuple(v if v else d for v, d in zip(c, _defaults(mode)))


def signature(groups: Sequence[B.GroupArgs], mode: int) -> str:
    """Shape signature of a call: per group its products' (D0, D1, D2,
    dtypes, transposes) and C's dtype, in call order, plus the mode."""
    parts = [f"mode={mode}"]
    for g in (groups.groups if isinstance(groups, B.GroupBatch) else groups):
        s = g.struct
        prods = []
        for k in range(s.n_prods):
            p = s.prods[k]
            prods.append(f"{p.D0}x{p.D1}x{p.D2}:{p.dtype_a}{p.dtype_b}:{p.trans_a}{p.trans_b}")
        parts.append(f"[{s.dtype_c};{','.join(prods)}]")
    return hashlib.sha256("|".join(parts).encode()).hexdigest()[:32]


class Planner:
    """Chooses and caches launch shapes per shape signature."""

    def __init__(self, cache_path: Optional[str] = None, grid=None, reps: int = 3):
        self.cache_path = cache_path
        self.grid = list(grid or DEFAULT_GRID)
        self.reps = reps
        self.cache: Dict[str, dict] = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    def _save(self):
        if not self.cache_path:
            return
        tmp = self.cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.cache, f, indent=1)
        os.replace(tmp, self.cache_path)

    @staticmethod
    def _tuning(rec: dict) -> "B.vl_tuning":
        return B.tuning(lane_macs=rec["lane_macs"], segments=rec["segments"], cols_rows=rec["cols_rows"],
                        claim_order=rec["claim_order"])

    def _time(self, groups, seed: int, mode: int, tun) -> float:
        import torch
        ws = torch.empty(max(256, B.workspace_size(groups, mode, tuning_=tun)), dtype=torch.uint8, device="cuda")
        B.sumcheck_matmul_prove(groups, seed, mode=mode, workspace=ws, tuning_=tun)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(self.reps):
            t0 = time.perf_counter()
            B.sumcheck_matmul_prove(groups, seed, mode=mode, workspace=ws, tuning_=tun)
            best = min(best, time.perf_counter() - t0)
        del ws
        return 1e3 * best

    def plan(self, groups: Sequence[B.GroupArgs], seed: int = 1, mode: int = B.VL_MODE_BATCHED) -> dict:
        """The cached record for this call's signature, tuned on a miss:
        {"lane_macs", "segments", "cols_rows", "claim_order", "ms",
        "default_ms", "grid"}."""
        key = signature(groups, mode)
        rec = self.cache.get(key)
        if rec is not None:
            return rec
        batch = groups if isinstance(groups, B.GroupBatch) else B.GroupBatch(list(groups))
        self._time(batch, seed, mode, None)      # first call of these shapes: warms caches and allocator
        # candidates that resolve to the defaults are the defaults; the
        # defaults and every other candidate are timed in two interleaved
        # passes (best of both), so drift over the sweep biases none of them
        cands = []
        for c in self.grid:
            r = _resolved(c, mode)
            if r != _defaults(mode) and r not in [_resolved(x, mode) for x in cands]:
                cands.append(c)
        times = {None: float("inf")}
        for c in cands:
            times[c] = float("inf")
        for _ in range(2):
            times[None] = min(times[None], self._time(batch, seed, mode, None))
            for c in cands:
                t = B.tuning(lane_macs=c[0], segments=c[1], cols_rows=c[2], claim_order=c[3])
                times[c] = min(times[c], self._time(batch, seed, mode, t))
        default_ms = times[None]
        table: List[dict] = [{"lane_macs": c[0], "segments": c[1], "cols_rows": c[2], "claim_order": c[3],
                              "ms": round(times[c], 4)} for c in cands]
        best = min(table, key=lambda r: r["ms"]) if table else None
        # the defaults unless a candidate is faster by more than the timing noise
        if best is None or best["ms"] >= 0.98 * default_ms:
            best = {"lane_macs": 0, "segments": 0, "cols_rows": 0, "claim_order": 0, "ms": round(default_ms, 4)}
        rec = dict(best)
        rec["default_ms"] = round(default_ms, 4)
        rec["grid"] = table
        self.cache[key] = rec
        self._save()
        return rec

    def tuning(self, groups: Sequence[B.GroupArgs], seed: int = 1, mode: int = B.VL_MODE_BATCHED):
        """vl_tuning for this call's shapes (tuned once per signature)."""
        return self._tuning(self.plan(groups, seed, mode))

    def lookup(self, groups: Sequence[B.GroupArgs], mode: int = B.VL_MODE_BATCHED):
        """The cached vl_tuning for these shapes, or None (never tunes: for
        paths that must not spend time timing candidates, such as a server's
        admission)."""
        rec = self.cache.get(signature(groups, mode))
        return None if rec is None else self._tuning(rec)
