"""Continuous-batching proof server (one GPU).

Proof requests (a list of groups with device-resident witnesses, and a seed)
arrive over time.  The server keeps a fixed number of slots; each slot owns a
HIP stream and pinned host buffers for proofs and status (kept across
requests and grown when a request needs more), and, while busy, a device
workspace.  A request is admitted when a slot is free and its device
memory (the workspace, plus its witness bytes if the caller says they are not
yet counted) fits the HBM budget; otherwise it waits in FIFO order.  Admitted
requests are enqueued with the asynchronous prove entry point, so requests on
different slots overlap on the device; the kernels write proof bytes and
status words straight into the pinned buffers (no copy-engine transfer, which
would order the slots' streams behind each other).  Completion is found by
polling HIP events, after which latency is recorded, the proof bytes are
copied out of the slot's pinned buffer and the slot and its device memory are
released.

The arithmetic is untouched: a request's proof bytes depend only on its
matrices, its seed and its group ids, so a result is identical alone and in
any mix (the serving tests check this).

Hardware queues: HIP gives each stream one of GPU_MAX_HW_QUEUES queues (4 by
default) at its first launch; slots whose streams share a queue run one
after the other there, one request's sumcheck rounds in front of the next
one's contractions.  A process serving n slots should set GPU_MAX_HW_QUEUES
to at least n + 2 before the GPU is first used (bench.py sets 16).
"""
import collections
import dataclasses
import time
from typing import Deque, Dict, List, Optional, Sequence

from . import binding as B


@dataclasses.dataclass
class Request:
    rid: int
    groups: Sequence[B.GroupArgs]
    seed: int
    t_arrive: float = 0.0
    witness_bytes: int = 0          # counted against the budget while in flight (0 = resident pool)
    mode: int = B.VL_MODE_BATCHED
    tuning: object = None           # vl_tuning; None: the server planner's cached choice, else defaults


@dataclasses.dataclass
class Result:
    rid: int
    proofs: List[bytes]
    status: List[int]
    t_arrive: float
    t_admit: float
    t_done: float

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrive


class _Slot:
    def __init__(self, torch, idx: int):
        self.idx = idx
        self.stream = torch.cuda.Stream()      # default priority
        self.req: Optional[Request] = None
        self.event = None
        self.bufs = None
        self.offs = None
        self.bytes = 0
        self.t_admit = 0.0
        self.host_proofs = None                # pinned, reused by the slot's requests
        self.host_status = None

    def host_buffers(self, torch, n_bytes: int, n_status: int):
        """Views of the slot's pinned buffers of at least the given sizes
        (reallocated only when a request needs more than any before it)."""
        if self.host_proofs is None or self.host_proofs.numel() < n_bytes:
            self.host_proofs = torch.empty(n_bytes, dtype=torch.uint8, pin_memory=True)
        if self.host_status is None or self.host_status.numel() < n_status:
            self.host_status = torch.empty(n_status, dtype=torch.int32, pin_memory=True)
        return self.host_proofs[:n_bytes], self.host_status[:n_status]


class ProofServer:
    def __init__(self, n_slots: int = 4, hbm_budget_bytes: int = 32 << 30, planner=None):
        import torch
        self.torch = torch
        self.planner = planner                 # tune.Planner: launch shapes per shape signature (cached only)
        self.slots = [_Slot(torch, i) for i in range(n_slots)]
        self.budget = hbm_budget_bytes
        self.in_use = 0
        self.queue: Deque[Request] = collections.deque()
        self.done: Dict[int, Result] = {}
        self.peak_in_flight = 0

    # -- sizing ---------------------------------------------------------------
    def _tuning(self, req: Request):
        if req.tuning is None and self.planner is not None:
            req.tuning = self.planner.lookup(req.groups, req.mode)
        return req.tuning

    def request_bytes(self, req: Request) -> int:
        """HBM bytes a request holds while in flight (its outputs are in host memory)."""
        return B.workspace_size(req.groups, req.mode, async_=True, tuning_=self._tuning(req)) + req.witness_bytes

    # -- queue ----------------------------------------------------------------
    def submit(self, req: Request):
        if req.mode == B.VL_MODE_PERSISTENT:
            # resident spinning rounds workgroups of several slots would hold
            # CUs and hardware queues that the other slots' contractions need
            raise ValueError("the server runs requests in batched mode; persistent mode is refused")
        if not req.t_arrive:
            req.t_arrive = time.perf_counter()
        if self.request_bytes(req) > self.budget:
            raise ValueError(f"request {req.rid} needs more than the whole HBM budget")
        self.queue.append(req)

    def _admit(self):
        torch = self.torch
        while self.queue:
            slot = next((s for s in self.slots if s.req is None), None)
            if slot is None:
                return
            req = self.queue[0]
            need = self.request_bytes(req)
            if self.in_use + need > self.budget:
                return                       # FIFO: wait for memory to free up
            self.queue.popleft()
            ng = len(req.groups)
            # the workspace comes from the slot's stream: freed when the slot
            # is released, its block is at once reusable by the slot's next
            # request (no cross-stream event, no new device allocation)
            tun = self._tuning(req)
            with torch.cuda.stream(slot.stream):
                ws = torch.empty(max(256, B.workspace_size(req.groups, req.mode, async_=True, tuning_=tun)),
                                 dtype=torch.uint8, device="cuda")
            total = sum(B.proof_size(g) for g in req.groups)
            # the slot is free, so nothing still writes its pinned buffers
            proofs, status = slot.host_buffers(torch, max(1, total), ng)
            status.numpy()[:] = -1
            # the slot's stream must see the witnesses made on the current stream
            slot.stream.wait_stream(torch.cuda.current_stream())
            slot.offs = B.sumcheck_matmul_prove_async(req.groups, req.seed, proofs, status, ws,
                                                      mode=req.mode, stream=slot.stream, tuning_=tun)
            ev = torch.cuda.Event()
            ev.record(slot.stream)
            slot.req, slot.event, slot.bufs, slot.bytes = req, ev, (ws, proofs, status), need
            slot.t_admit = time.perf_counter()
            self.in_use += need
            self.peak_in_flight = max(self.peak_in_flight, sum(s.req is not None for s in self.slots))

    def _reap(self) -> int:
        n = 0
        for s in self.slots:
            if s.req is None or not s.event.query():
                continue
            ws, proofs, status = s.bufs
            # numpy views of the pinned buffers: no torch CPU op (its thread
            # pool would compete with the next admission's host work)
            raw = proofs.numpy().tobytes()
            st = status.numpy().tolist()
            req = s.req
            self.done[req.rid] = Result(req.rid, [raw[s.offs[i]:s.offs[i + 1]] for i in range(len(req.groups))],
                                        st, req.t_arrive, s.t_admit, time.perf_counter())
            self.in_use -= s.bytes
            s.req = s.event = s.bufs = s.offs = None
            s.bytes = 0
            n += 1
        return n

    def poll(self) -> int:
        """Admit what fits, collect what finished; returns requests completed."""
        n = self._reap()
        self._admit()
        return n

    def busy(self) -> bool:
        return bool(self.queue) or any(s.req is not None for s in self.slots)

    def drain(self, sleep_s: float = 0.0):
        while self.busy():
            if self.poll() == 0 and sleep_s:
                time.sleep(sleep_s)


def run_open_loop(server: ProofServer, arrivals, make_request, sleep_s: float = 0.00005):
    """Feed requests at their arrival times (seconds from start) and run the
    server until all are done.  ``arrivals`` is a list of (t, payload);
    ``make_request(i, payload)`` returns a Request.  Returns the results in
    arrival order and the wall time."""
    t0 = time.perf_counter()
    i = 0
    while i < len(arrivals) or server.busy():
        now = time.perf_counter() - t0
        while i < len(arrivals) and arrivals[i][0] <= now:
            req = make_request(i, arrivals[i][1])
            req.t_arrive = t0 + arrivals[i][0]
            server.submit(req)
            i += 1
        if server.poll() == 0 and sleep_s:
            time.sleep(sleep_s)
    wall = time.perf_counter() - t0
    return [server.done[k] for k in sorted(server.done)], wall


def latency_summary(results: Sequence[Result]) -> dict:
    lat = sorted(r.latency for r in results)
    if not lat:
        return {}
    pick = lambda q: lat[min(len(lat) - 1, max(0, int(round(q * len(lat))) - 1))]  # noqa: E731
    return {"p50_ms": 1e3 * pick(0.50), "p99_ms": 1e3 * pick(0.99), "mean_ms": 1e3 * sum(lat) / len(lat),
            "n": len(lat)}
