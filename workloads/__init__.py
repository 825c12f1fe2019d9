"""Seeded synthetic workloads for the matmul-sumcheck prover.

This package only draws integer tensors and forms the witness products that a
prover is asked to prove; it holds none of the proof system's arithmetic (no
field, no multilinear extension, no transcript).  Both the CPU oracle
(``oracle/``) and the device library's tests and benchmark take their inputs
from here, so the two sides see identical bytes.
"""
from .gen import (  # noqa: F401
    Product, Group, Workload,
    quantize_gaussian, requant, exact_matmul,
    config1, lora_forward, lora_backward_update, config2, config3, config4,
    LayerWitness, layer_witness, chain_layer, tiny_layer, CHAIN_F, CHAIN_ETA,
    serving_request, serving_stream, frozen_weight, serving_sample, serving_sample_workload, tiny_random_group, CONFIG_NAMES, make_config,
    HeadView, HeadBatch, cols_heads, stacked_heads, attention_layer, tiny_head_batch,
    LookupCase, silu_table, lookup_range, lookup_silu, tiny_lookup, block_weights,
)
