"""Chained proof of one LoRA layer's step against the oracle (needs a gfx950 GPU).

vl_lora_chain_prove must write exactly the oracle's bytes (oracle/chain.py):
tiny layers against the full proofs in tests/golden/chain.json, and the
FFN-up layer of the backward-and-update configuration (T = 512,
4096 -> 11008, rank 16) against its stored digest.  That layer's chain
covers the update checks of A and B, the forward and dX sum groups, and the
reduction of the three claims on X (from X W, X A and X^T G) to one.
"""
import sys

import numpy as np
import pytest

import workloads
from gpu_util import golden, sha, to_dev

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_21393_amd import binding
    binding.lib()
    return binding


class _Dev:
    """A LayerWitness with every tensor copied to the device."""

    def __init__(self, w):
        for n in ("X", "W", "A", "B", "dY", "H", "G", "Y", "C2", "C4", "dA", "dB", "dX", "UA", "UB"):
            setattr(self, n, to_dev(getattr(w, n)))
        self.F, self.eta = w.F, w.eta


def test_chain_tiny_layers_match_oracle_bytes(B):
    gold = golden("chain")
    for rec in gold["tiny"]:
        seed, T, d_in, d_out, r = rec["spec"]
        _say(f"chain tiny layer T={T} d_in={d_in} d_out={d_out} r={r}")
        w = workloads.tiny_layer(seed, T, d_in, d_out, r)
        proof, dig = B.lora_chain_prove(B.LayerArgs(_Dev(w)), gold["seed"])
        assert proof.hex() == rec["proof_hex"], rec["spec"]
        assert dig.hex() == rec["state"], rec["spec"]


def test_chain_full_size_ffn_up_layer_matches_oracle(B):
    gold = golden("chain")["layer"]
    _say("chain FFN-up layer: generating")
    w = workloads.chain_layer(device="cuda")
    assert list(w.dims) == gold["dims"]
    _say("chain FFN-up layer: proving")
    la = B.LayerArgs(_Dev(w))
    proof, dig = B.lora_chain_prove(la, golden("chain")["seed"])
    assert len(proof) == gold["proof_len"]
    assert sha(proof) == gold["proof_sha256"]
    assert dig.hex() == gold["state"]
    _say("chain FFN-up layer: second proof, same workspace")
    proof2, _ = B.lora_chain_prove(la, golden("chain")["seed"])
    assert proof2 == proof


@pytest.mark.parametrize("name", ["UA", "dA", "Y", "dX", "C4"])
def test_chain_refuses_false_statements(B, name):
    w = workloads.tiny_layer(7, 4, 6, 5, 2)
    M = getattr(w, name).copy()
    M[0, 0] += 1
    setattr(w, name, M)
    if name == "dA":   # keep the update relation true for the wrong gradient
        w.UA = (w.A.astype(np.int64) << w.F) - w.eta * M
    _say(f"chain false statement in {name}")
    with pytest.raises(B.VLError) as e:
        B.lora_chain_prove(B.LayerArgs(_Dev(w)), 1)
    assert e.value.status == B.VL_ERR_FALSE_STATEMENT
