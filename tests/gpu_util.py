"""Helpers for GPU tests: move seeded workloads to the device as GroupArgs."""
import hashlib
import json
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden")


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def device_group(g, B):
    """workloads.Group -> binding.GroupArgs over device copies of its tensors."""
    prods = [(to_dev(p.A), to_dev(p.B), p.transA, p.transB) for p in g.products]
    return B.GroupArgs(g.group_id, prods, to_dev(g.C))


def golden(name):
    with open(os.path.join(GOLD, f"{name}.json")) as f:
        return json.load(f)


def sha(b: bytes) -> str:
    return hashlib.sha256(b).hexdigest()


def tiny_workload():
    import workloads
    spec = golden("tiny")
    groups = []
    for k, (seed, dims, dt, trans, vb) in enumerate(spec["tiny_spec"]):
        g = workloads.tiny_random_group(seed, [tuple(d) for d in dims], dtype=getattr(np, dt),
                                        trans=tuple(trans), value_bits=vb, name=f"tiny{k}")
        g.group_id = k
        groups.append(g)
    return workloads.Workload(spec["workload"], spec["seed"], groups), spec
