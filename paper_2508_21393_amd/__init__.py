"""MI355X (gfx950) prover for matrix-multiplication sumcheck claims.

Proves C = A.B (and sums of products) over the BLS12-381 scalar field with the
sumcheck protocol of the paper's Sec. II-C, as zkMat does for every matmul of
a LoRA fine-tuning step (Sec. IV-B).  The work runs in the HIP kernels of
``libverilora.so`` behind the C ABI of ``include/verilora.h``; this package is
a thin ctypes binding plus the batching and serving layers.
"""
from . import binding  # noqa: F401
from .binding import (  # noqa: F401
    GroupArgs, VLError, fr_lift, fr_export, eq_table, mle_partial_eval, partial_eval_workspace_size,
    proof_size, workspace_size, sumcheck_matmul_prove, sumcheck_matmul_prove_async, verify_transcript,
    VL_MODE_PER_INSTANCE, VL_MODE_BATCHED, VL_MODE_PERSISTENT, VL_CONTRACT_ROWS, VL_CONTRACT_COLS,
)
