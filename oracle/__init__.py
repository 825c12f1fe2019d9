"""CPU oracle for the matmul sumcheck (test infrastructure, not product code).

A plain, slow and obviously correct restatement of what the prover computes,
written from the paper's definitions in Python integers:

  * ``field``      -- the prime field (BLS12-381 scalar field, a choice of this
                      project; the paper only asks for |F| ~ 2^254, Sec. V).
  * ``transcript`` -- the Fiat-Shamir transcript (Sec. IV-A footnote on
                      Fiat-Shamir; Sec. II-B.1), on hashlib's SHA-256.
  * ``mle``        -- multilinear extensions and the Lagrange basis eq(x, b)
                      exactly as in eq. (MLE), Sec. II-B.2.
  * ``zkmat``      -- the matmul sumcheck of eq. (zk-mle-matmul), Sec. II-C,
                      prover and verifier, as used by zkMat (Sec. IV-B).

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package.  The device library never does,
and this package imports nothing from it; the two share only the seeded input
generators in ``workloads/``.
"""
from .field import P, lift, enc, dec, inv  # noqa: F401
from .transcript import Transcript, sha256  # noqa: F401
from .mle import num_vars, bits_msb_first, eq_basis, eq_table, mle_eval, matrix_mle  # noqa: F401
from .mle import partial_eval_rows, partial_eval_cols  # noqa: F401
from .zkmat import (  # noqa: F401
    prove_group, verify_group, FalseStatement, Reject, ProofParts, claim_value,
    round_poly, interpolate_quadratic,
)
