"""ctypes binding of libverilora.so (argument marshalling only).

The functions below carry the C ABI's names (without the ``vl_`` prefix) and
pass raw pointers through; every step of the prover runs in the library's
HIP kernels.  PyTorch supplies device memory and the current HIP stream.  If
the library has not been built the first call raises: there is no fallback.
"""
import ctypes
import os
from typing import List, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libverilora.so")

VL_OK, VL_ERR_INVALID_ARG, VL_ERR_SHAPE, VL_ERR_DTYPE, VL_ERR_WORKSPACE, VL_ERR_HIP, \
    VL_ERR_FALSE_STATEMENT, VL_ERR_REJECT, VL_ERR_BUFFER_TOO_SMALL, VL_ERR_RANGE, VL_ERR_TIMEOUT = range(11)
VL_I16, VL_I32, VL_I64 = 1, 2, 3
VL_CONTRACT_ROWS, VL_CONTRACT_COLS = 0, 1
VL_MODE_PER_INSTANCE, VL_MODE_BATCHED, VL_MODE_PERSISTENT = 0, 1, 2
VL_MAX_PRODS = 8
VL_STAGE_COUNT = 24
STAGE_NAMES = ["upload", "eq", "i16_rows", "i16_rows4", "i16_rows4_vec", "i16_cols", "i16_cols_vec",
               "i16_cols2_vec", "i32_rows", "i32_rows4_vec", "i32_cols", "i32_cols_vec", "i64s_rows",
               "i64s_rows2_vec", "i64s_cols", "i64s_cols_vec", "i64s_cols2_vec", "i64_rows", "i64_rows2_vec",
               "i64_cols", "i64_cols_vec", "finish", "pass1", "rounds"]

STATUS_NAMES = {0: "VL_OK", 1: "VL_ERR_INVALID_ARG", 2: "VL_ERR_SHAPE", 3: "VL_ERR_DTYPE",
                4: "VL_ERR_WORKSPACE", 5: "VL_ERR_HIP", 6: "VL_ERR_FALSE_STATEMENT",
                7: "VL_ERR_REJECT", 8: "VL_ERR_BUFFER_TOO_SMALL", 9: "VL_ERR_RANGE", 10: "VL_ERR_TIMEOUT"}

EXPORTED = ("vl_fr_lift", "vl_fr_export", "vl_eq_table", "vl_partial_eval_workspace_size",
            "vl_mle_partial_eval", "vl_proof_size", "vl_workspace_size",
            "vl_sumcheck_matmul_prove", "vl_verify_transcript", "vl_last_error",
            "vl_prove_graph_create", "vl_prove_graph_launch", "vl_prove_graph_bind", "vl_prove_graph_destroy",
            "vl_mle_partial_eval_noalloc", "vl_lora_chain_proof_size", "vl_lora_chain_workspace_size",
            "vl_lora_chain_prove", "vl_bmm_proof_size", "vl_bmm_workspace_size", "vl_bmm_prove",
            "vl_bmm_verify", "vl_lookup_proof_size", "vl_lookup_workspace_size", "vl_lookup_prove",
            "vl_lookup_verify", "vl_hyrax_table_size", "vl_hyrax_setup", "vl_hyrax_commit_workspace_size",
            "vl_hyrax_commit", "vl_hyrax_generators", "vl_hyrax_verify_open")
NOALLOC_SCRATCH_BYTES = 64 << 20   # VL_NOALLOC_SCRATCH_BYTES
# the library's field Fr: the BLS12-381 scalar field (for drawing points)
FR_MODULUS = 0x73eda753299d7d483339d80809a1d80553bda402fffe5bfeffffffff00000001

c_u32, c_u64, c_i32, c_vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p


class vl_fr(ctypes.Structure):
    _fields_ = [("w", c_u32 * 8)]


class vl_fr_vec(ctypes.Structure):
    _fields_ = [("base", c_vp), ("n", c_u64), ("ld", c_u64)]


class vl_product(ctypes.Structure):
    _fields_ = [("A", c_vp), ("B", c_vp), ("dtype_a", c_i32), ("dtype_b", c_i32),
                ("D0", c_u32), ("D1", c_u32), ("D2", c_u32), ("lda", c_u64), ("ldb", c_u64),
                ("trans_a", c_i32), ("trans_b", c_i32)]


class vl_group(ctypes.Structure):
    _fields_ = [("prods", ctypes.POINTER(vl_product)), ("n_prods", c_u32), ("group_id", c_u32),
                ("C", c_vp), ("dtype_c", c_i32), ("ldc", c_u64), ("bind", c_vp)]


class vl_tuning(ctypes.Structure):
    _fields_ = [("lane_macs", c_u32), ("min_tasks", c_u32), ("segments", c_u32), ("cols_rows", c_u32),
                ("spin_limit", c_u32), ("claim_order", c_u32), ("contract_streams", c_u32)]


def tuning(lane_macs: int = 0, min_tasks: int = 0, segments: int = 0, cols_rows: int = 0,
           spin_limit: int = 0, claim_order: int = 0, contract_streams: int = 0) -> vl_tuning:
    """Launch-shape knobs (0 = library default); results never depend on them
    (a spin limit too small for the work makes persistent-mode groups fail
    with VL_ERR_TIMEOUT instead)."""
    return vl_tuning(lane_macs, min_tasks, segments, cols_rows, spin_limit, claim_order, contract_streams)


def _tun(t):
    return ctypes.pointer(t) if t is not None else None


class vl_prove_opts(ctypes.Structure):
    _fields_ = [("mode", c_i32), ("async_", c_i32), ("workspace", c_vp), ("workspace_bytes", c_u64),
                ("status", c_vp), ("tuning", ctypes.POINTER(vl_tuning)), ("stage_ms", c_vp)]


class vl_lora_layer(ctypes.Structure):
    _fields_ = [("T", c_u32), ("d_in", c_u32), ("d_out", c_u32), ("r", c_u32), ("F", c_u32), ("eta", c_u32)] + \
        [(n, c_vp) for n in ("X", "W", "A", "B", "dY", "H", "G", "Y", "C2", "C4", "dA", "dB", "dX", "UA", "UB")]


class vl_bmm(ctypes.Structure):
    _fields_ = [("A", c_vp), ("B", c_vp), ("C", c_vp), ("dtype_a", c_i32), ("dtype_b", c_i32), ("dtype_c", c_i32),
                ("H", c_u32), ("D0", c_u32), ("D1", c_u32), ("D2", c_u32), ("lda", c_u64), ("ldb", c_u64),
                ("ldc", c_u64), ("head_stride_a", c_u64), ("head_stride_b", c_u64), ("head_stride_c", c_u64),
                ("trans_a", c_i32), ("trans_b", c_i32), ("group_id", c_u32)]


class vl_lookup(ctypes.Structure):
    _fields_ = [("x", c_vp), ("y", c_vp), ("tb", c_vp), ("dtype", c_i32), ("dtype_y", c_i32), ("t0", c_i32),
                ("two_col", c_i32), ("N", c_u32), ("D", c_u64), ("id", c_u32)]


LAYER_INT16 = ("X", "W", "A", "B", "dY", "H", "G")
LAYER_INT64 = ("Y", "C2", "C4", "dA", "dB", "dX", "UA", "UB")


class VLError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2508_21393_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.vl_fr_lift.argtypes = [c_vp, c_i32, c_u64, vl_fr_vec, c_vp]
        L.vl_fr_export.argtypes = [vl_fr_vec, c_u64, c_vp, c_vp]
        L.vl_eq_table.argtypes = [ctypes.POINTER(vl_fr), c_u32, vl_fr_vec, c_vp]
        L.vl_partial_eval_workspace_size.argtypes = [c_u32, c_u32, c_i32, c_i32, ctypes.POINTER(vl_tuning)]
        L.vl_partial_eval_workspace_size.restype = c_u64
        L.vl_mle_partial_eval.argtypes = [c_vp, c_i32, c_u32, c_u32, c_u64, c_i32, vl_fr_vec, vl_fr_vec,
                                          c_vp, c_u64, ctypes.POINTER(vl_tuning), c_vp]
        L.vl_mle_partial_eval_noalloc.argtypes = [c_vp, c_i32, c_u32, c_u32, c_u64, c_i32, vl_fr_vec, vl_fr_vec,
                                                  ctypes.POINTER(vl_tuning), c_vp]
        L.vl_lora_chain_proof_size.argtypes = [ctypes.POINTER(vl_lora_layer)]
        L.vl_lora_chain_proof_size.restype = c_u64
        L.vl_lora_chain_workspace_size.argtypes = [ctypes.POINTER(vl_lora_layer)]
        L.vl_lora_chain_workspace_size.restype = c_u64
        L.vl_lora_chain_prove.argtypes = [ctypes.POINTER(vl_lora_layer), c_u64, c_vp, c_u64, c_vp, c_u64, c_vp, c_vp]
        L.vl_lora_chain_prove.restype = c_i32
        L.vl_proof_size.argtypes = [ctypes.POINTER(vl_group)]
        L.vl_proof_size.restype = c_u64
        L.vl_workspace_size.argtypes = [ctypes.POINTER(vl_group), c_u64, ctypes.POINTER(vl_prove_opts)]
        L.vl_workspace_size.restype = c_u64
        L.vl_sumcheck_matmul_prove.argtypes = [ctypes.POINTER(vl_group), c_u64, c_u64,
                                               ctypes.POINTER(vl_prove_opts), c_vp, c_u64,
                                               ctypes.POINTER(c_u64), c_vp, c_vp]
        L.vl_verify_transcript.argtypes = [c_vp, c_u64, ctypes.POINTER(vl_group), c_u64,
                                           ctypes.POINTER(vl_fr), c_u64, ctypes.POINTER(c_u64),
                                           ctypes.POINTER(c_i32)]
        L.vl_last_error.restype = ctypes.c_char_p
        L.vl_bmm_proof_size.argtypes = [ctypes.POINTER(vl_bmm)]
        L.vl_bmm_proof_size.restype = c_u64
        L.vl_bmm_workspace_size.argtypes = [ctypes.POINTER(vl_bmm), c_u64]
        L.vl_bmm_workspace_size.restype = c_u64
        L.vl_bmm_prove.argtypes = [ctypes.POINTER(vl_bmm), c_u64, c_u64, c_vp, c_u64, c_vp, c_u64,
                                   ctypes.POINTER(c_u64), c_vp, c_vp]
        L.vl_bmm_prove.restype = c_i32
        L.vl_bmm_verify.argtypes = [c_vp, c_u64, ctypes.POINTER(vl_bmm), c_u64, ctypes.POINTER(vl_fr), c_u64,
                                    ctypes.POINTER(c_u64), ctypes.POINTER(c_i32)]
        L.vl_bmm_verify.restype = c_i32
        L.vl_lookup_proof_size.argtypes = [ctypes.POINTER(vl_lookup)]
        L.vl_lookup_proof_size.restype = c_u64
        L.vl_lookup_workspace_size.argtypes = [ctypes.POINTER(vl_lookup), c_u64]
        L.vl_lookup_workspace_size.restype = c_u64
        L.vl_lookup_prove.argtypes = [ctypes.POINTER(vl_lookup), c_u64, c_u64, c_vp, c_u64, c_vp, c_u64,
                                      ctypes.POINTER(c_u64), c_vp, c_vp]
        L.vl_lookup_prove.restype = c_i32
        L.vl_lookup_verify.argtypes = [c_vp, c_u64, ctypes.POINTER(vl_lookup), c_u64, ctypes.POINTER(vl_fr), c_u64,
                                       ctypes.POINTER(c_u64), ctypes.POINTER(c_i32)]
        L.vl_lookup_verify.restype = c_i32
        L.vl_hyrax_table_size.argtypes = [c_u32, c_u32]
        L.vl_hyrax_table_size.restype = c_u64
        L.vl_hyrax_setup.argtypes = [c_u32, c_u32, c_vp, c_u64, c_vp]
        L.vl_hyrax_setup.restype = c_i32
        L.vl_hyrax_commit_workspace_size.argtypes = [c_u32, c_u32, c_u32]
        L.vl_hyrax_commit_workspace_size.restype = c_u64
        L.vl_hyrax_commit.argtypes = [c_vp, c_i32, c_u32, c_u32, c_u64, c_vp, c_u32, c_u32, c_u32, c_vp, c_vp, c_u64,
                                      c_vp]
        L.vl_hyrax_commit.restype = c_i32
        L.vl_hyrax_generators.argtypes = [c_u32, c_vp]
        L.vl_hyrax_generators.restype = c_i32
        L.vl_hyrax_verify_open.argtypes = [c_vp, c_u32, c_u32, ctypes.POINTER(vl_fr), ctypes.POINTER(vl_fr),
                                           ctypes.POINTER(vl_fr), ctypes.POINTER(vl_fr)]
        L.vl_hyrax_verify_open.restype = c_i32
        L.vl_prove_graph_create.argtypes = [ctypes.POINTER(vl_group), c_u64, ctypes.POINTER(vl_prove_opts), c_vp,
                                            c_u64, ctypes.POINTER(c_u64), c_vp, ctypes.POINTER(c_vp)]
        L.vl_prove_graph_launch.argtypes = [c_vp, c_u64, c_vp]
        L.vl_prove_graph_bind.argtypes = [c_vp, c_vp]
        L.vl_prove_graph_destroy.argtypes = [c_vp]
        L.vl_prove_graph_destroy.restype = None
        for f in ("vl_fr_lift", "vl_fr_export", "vl_eq_table", "vl_mle_partial_eval", "vl_mle_partial_eval_noalloc",
                  "vl_sumcheck_matmul_prove", "vl_verify_transcript", "vl_prove_graph_create",
                  "vl_prove_graph_launch", "vl_prove_graph_bind"):
            getattr(L, f).restype = c_i32
        _lib = L
    return _lib


def last_error() -> str:
    return lib().vl_last_error().decode()


def _check(status: int):
    if status != VL_OK:
        raise VLError(status, last_error())


# ---------------------------------------------------------------- helpers ----
def dtype_code(dt) -> int:
    """VL_I16/I32/I64 for a torch dtype, a numpy dtype or a numpy scalar type."""
    s = str(dt).replace("torch.", "")
    if s not in ("int16", "int32", "int64"):
        import numpy as np
        s = np.dtype(dt).name
    return {"int16": VL_I16, "int32": VL_I32, "int64": VL_I64}[s]


def _ptr(x) -> int:
    """Raw pointer of a torch tensor (device or host) or a numpy array (host)."""
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    return x.ctypes.data


def _row_stride(x) -> int:
    """Leading dimension in elements (a single row may report any stride)."""
    rows, cols = x.shape
    if hasattr(x, "stride") and callable(x.stride):
        assert cols <= 1 or x.stride(1) == 1, "matrices must be row-major"
        ld = x.stride(0)
    else:
        assert cols <= 1 or x.strides[1] == x.itemsize, "matrices must be row-major"
        ld = x.strides[0] // x.itemsize
    return ld if rows > 1 else max(ld, cols, 1)


def fr_to_int(f: vl_fr) -> int:
    return sum(int(f.w[i]) << (32 * i) for i in range(8))


def int_to_fr(x: int) -> vl_fr:
    f = vl_fr()
    for i in range(8):
        f.w[i] = (x >> (32 * i)) & 0xFFFFFFFF
    return f


def fr_vec(t, n: Optional[int] = None) -> vl_fr_vec:
    """A (8, ld) uint32/int32 device tensor viewed as a structure-of-limbs vector."""
    assert t.dim() == 2 and t.shape[0] == 8 and t.stride(1) == 1
    return vl_fr_vec(t.data_ptr(), t.shape[1] if n is None else n, t.stride(0))


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _bind_buffer(bind):
    """A 32-byte host buffer holding a bind digest (None stays None)."""
    if bind is None:
        return None
    bind = bytes(bind)
    if len(bind) != 32:
        raise ValueError("a bind digest is 32 bytes")
    return ctypes.create_string_buffer(bind, 32)


class GroupArgs:
    """vl_group built from (A, B, transA, transB) operands and C, with an
    optional 32-byte bind digest of the caller's commitments; keeps the
    Python objects alive as long as the structure is used."""

    def __init__(self, group_id: int, prods: Sequence[Tuple[object, object, bool, bool]], C, bind=None):
        self.keep = [C] + [x for p in prods for x in p[:2]]
        self._bind = _bind_buffer(bind)
        arr = (vl_product * len(prods))()
        for k, (A, B, ta, tb) in enumerate(prods):
            a_rows, a_cols = A.shape
            b_rows, b_cols = B.shape
            D0, D1 = (a_cols, a_rows) if ta else (a_rows, a_cols)
            D1b, D2 = (b_cols, b_rows) if tb else (b_rows, b_cols)
            assert D1 == D1b, "inner dimensions differ"
            arr[k] = vl_product(_ptr(A), _ptr(B), dtype_code(A.dtype), dtype_code(B.dtype), D0, D1, D2,
                                _row_stride(A), _row_stride(B), int(ta), int(tb))
        self.prods = arr
        self.struct = vl_group(arr, len(prods), group_id, _ptr(C), dtype_code(C.dtype), _row_stride(C),
                               ctypes.addressof(self._bind) if self._bind is not None else None)

    @classmethod
    def shapes_only(cls, group_id: int, shapes: Sequence[Tuple[int, int, int]], dtype_a="int16",
                    dtype_b="int16", dtype_c="int64", bind=None) -> "GroupArgs":
        """A group of the given (D0, D1, D2) products with no matrices (NULL
        pointers, plain layouts): for the verifier without a witness, whose
        reduced claims are then checked by commitment openings."""
        g = cls.__new__(cls)
        g.keep = []
        g._bind = _bind_buffer(bind)
        arr = (vl_product * len(shapes))()
        for k, (D0, D1, D2) in enumerate(shapes):
            arr[k] = vl_product(None, None, dtype_code(dtype_a), dtype_code(dtype_b), D0, D1, D2, D1, D2, 0, 0)
        g.prods = arr
        g.struct = vl_group(arr, len(shapes), group_id, None, dtype_code(dtype_c), shapes[0][2],
                            ctypes.addressof(g._bind) if g._bind is not None else None)
        return g

    @property
    def shapes(self):
        return [(p.D0, p.D1, p.D2) for p in self.prods]


def group_array(groups: Sequence[GroupArgs]):
    arr = (vl_group * len(groups))()
    for i, g in enumerate(groups):
        arr[i] = g.struct
    return arr


class GroupBatch:
    """The vl_group array of a list of groups with their proof sizes, built
    once and reusable for any number of prove calls over the same operand
    buffers (their contents may change between calls)."""

    def __init__(self, groups: Sequence[GroupArgs]):
        self.groups = list(groups)
        self.arr = group_array(self.groups)
        self.sizes = [proof_size(g) for g in self.groups]
        self.total = sum(self.sizes)
        self._ws = {}

    def __len__(self):
        return len(self.groups)

    def workspace_size(self, mode: int, async_: bool = False, tuning_=None) -> int:
        key = (mode, bool(async_), None if tuning_ is None else bytes(tuning_))
        if key not in self._ws:
            opts = vl_prove_opts(mode, int(async_), None, 0, None, _tun(tuning_), None)
            self._ws[key] = lib().vl_workspace_size(self.arr, len(self.groups), ctypes.byref(opts))
        return self._ws[key]


def _batch(groups) -> GroupBatch:
    return groups if isinstance(groups, GroupBatch) else GroupBatch(groups)


# ---------------------------------------------------------------- the ABI ----
def fr_lift(src, n: int, dst: vl_fr_vec, stream=None):
    _check(lib().vl_fr_lift(_ptr(src), dtype_code(src.dtype), n, dst, _stream(stream)))


def fr_export(src: vl_fr_vec, n: int, dst, stream=None):
    _check(lib().vl_fr_export(src, n, _ptr(dst), _stream(stream)))


def eq_table(point: Sequence[int], out: vl_fr_vec, stream=None):
    arr = (vl_fr * max(1, len(point)))(*[int_to_fr(x) for x in point])
    _check(lib().vl_eq_table(arr, len(point), out, _stream(stream)))


def partial_eval_workspace_size(rows: int, cols: int, contract: int, dtype, tuning_=None) -> int:
    return lib().vl_partial_eval_workspace_size(rows, cols, contract, dtype_code(dtype), _tun(tuning_))


def mle_partial_eval(M, contract: int, eq: vl_fr_vec, out: vl_fr_vec, workspace, stream=None, tuning_=None):
    rows, cols = M.shape
    _check(lib().vl_mle_partial_eval(_ptr(M), dtype_code(M.dtype), rows, cols, _row_stride(M), contract,
                                     eq, out, _ptr(workspace), workspace.numel() * workspace.element_size(),
                                     _tun(tuning_), _stream(stream)))


def mle_partial_eval_noalloc(M, contract: int, eq: vl_fr_vec, out: vl_fr_vec, stream=None, tuning_=None):
    """mle_partial_eval with the library's fixed device scratch (no workspace,
    no allocation); calls overlapping on one GPU race on that scratch."""
    rows, cols = M.shape
    _check(lib().vl_mle_partial_eval_noalloc(_ptr(M), dtype_code(M.dtype), rows, cols, _row_stride(M), contract,
                                             eq, out, _tun(tuning_), _stream(stream)))


def proof_size(group: GroupArgs) -> int:
    return lib().vl_proof_size(ctypes.byref(group.struct))


def workspace_size(groups, mode: int = VL_MODE_BATCHED, async_: bool = False, tuning_=None) -> int:
    """Workspace bytes for a list of GroupArgs or a GroupBatch."""
    return _batch(groups).workspace_size(mode, async_, tuning_)


def sumcheck_matmul_prove(groups, seed: int, mode: int = VL_MODE_BATCHED,
                          workspace=None, stream=None, with_digests: bool = True, stage_ms=None,
                          tuning_=None):
    """Blocking prove of a list of GroupArgs (or a GroupBatch): returns
    (list of proof bytes, list of 32-byte digests).

    ``stage_ms``: optional list that receives VL_STAGE_COUNT per-stage device
    times (HIP events) of this call.  ``tuning_``: optional vl_tuning."""
    import torch
    batch = _batch(groups)
    n = len(batch)
    if workspace is None:
        ws_bytes = batch.workspace_size(mode, False, tuning_)
        workspace = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device="cuda")
    timing = (ctypes.c_float * VL_STAGE_COUNT)() if stage_ms is not None else None
    opts = vl_prove_opts(mode, 0, workspace.data_ptr(), workspace.numel(), None, _tun(tuning_),
                         ctypes.addressof(timing) if timing is not None else None)
    total = batch.total
    buf = ctypes.create_string_buffer(max(total, 1))
    offs = (c_u64 * (n + 1))()
    dig = ctypes.create_string_buffer(32 * n) if with_digests else None
    _check(lib().vl_sumcheck_matmul_prove(batch.arr, n, seed, ctypes.byref(opts), ctypes.addressof(buf), total,
                                          offs, ctypes.addressof(dig) if dig is not None else None,
                                          _stream(stream)))
    if timing is not None:
        stage_ms[:] = list(timing)
    raw = buf.raw
    proofs = [raw[offs[i]:offs[i + 1]] for i in range(n)]
    digests = [dig.raw[32 * i:32 * i + 32] for i in range(n)] if dig is not None else None
    return proofs, digests


def sumcheck_matmul_prove_async(groups: Sequence[GroupArgs], seed: int, proofs_dev, status_dev,
                                workspace, mode: int = VL_MODE_BATCHED, digests_dev=None, stream=None,
                                tuning_=None):
    """Enqueue a prove on the stream; proofs/status/digests land in device
    tensors or pinned host tensors (written by the kernels, no copy).
    Returns the host offsets of each group's proof."""
    batch = _batch(groups)
    n = len(batch)
    opts = vl_prove_opts(mode, 1, workspace.data_ptr(), workspace.numel(), status_dev.data_ptr(),
                         _tun(tuning_), None)
    offs = (c_u64 * (n + 1))()
    _check(lib().vl_sumcheck_matmul_prove(batch.arr, n, seed, ctypes.byref(opts), proofs_dev.data_ptr(),
                                          proofs_dev.numel(), offs,
                                          digests_dev.data_ptr() if digests_dev is not None else None,
                                          _stream(stream)))
    return [int(offs[i]) for i in range(n + 1)]


class ProveGraph:
    """vl_prove_graph: the batched prove of these groups captured once into a
    HIP graph, with the workspace and output buffers fixed (device or pinned
    host tensors).  launch(seed, stream) proves the groups' current
    contents; close() (or the context manager) releases the graph."""

    def __init__(self, groups: Sequence[GroupArgs], workspace, proofs_dev, status_dev, mode: int = VL_MODE_BATCHED,
                 digests_dev=None, tuning_=None):
        self.batch = _batch(groups)
        n = len(self.batch)
        # the tensors must outlive the graph: keep references
        self._keep = (workspace, proofs_dev, status_dev, digests_dev, tuning_)
        self._tun = _tun(tuning_)
        self.opts = vl_prove_opts(mode, 1, workspace.data_ptr(), workspace.numel(), status_dev.data_ptr(),
                                  self._tun, None)
        offs = (c_u64 * (n + 1))()
        h = c_vp()
        _check(lib().vl_prove_graph_create(self.batch.arr, n, ctypes.byref(self.opts), proofs_dev.data_ptr(),
                                           proofs_dev.numel(), offs,
                                           digests_dev.data_ptr() if digests_dev is not None else None,
                                           ctypes.byref(h)))
        self.handle = h
        self.offsets = [int(offs[i]) for i in range(n + 1)]

    def launch(self, seed: int, stream=None):
        _check(lib().vl_prove_graph_launch(self.handle, seed, _stream(stream)))

    def bind(self, binds=None):
        """New bind digests for the next launches: None, or one 32-byte
        digest per group in the order given at create."""
        if binds is None:
            _check(lib().vl_prove_graph_bind(self.handle, None))
            return
        raw = b"".join(bytes(b) for b in binds)
        if len(raw) != 32 * len(self.batch):
            raise ValueError("one 32-byte digest per group")
        buf = ctypes.create_string_buffer(raw, len(raw))
        _check(lib().vl_prove_graph_bind(self.handle, ctypes.addressof(buf)))

    def close(self):
        if self.handle is not None and self.handle.value:
            lib().vl_prove_graph_destroy(self.handle)
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LayerArgs:
    """vl_lora_layer over a layer's tensors (objects with the attributes of
    LAYER_INT16 and LAYER_INT64, and F, eta: device tensors for proving),
    kept alive as long as the structure is used."""

    def __init__(self, w):
        self.keep = [getattr(w, n) for n in LAYER_INT16 + LAYER_INT64]
        T, d_in = w.X.shape
        d_out, r = w.W.shape[1], w.A.shape[1]
        for n in LAYER_INT16:
            assert dtype_code(getattr(w, n).dtype) == VL_I16, n
        for n in LAYER_INT64:
            assert dtype_code(getattr(w, n).dtype) == VL_I64, n
        for x in self.keep:
            rows, cols = x.shape
            assert _row_stride(x) == max(cols, 1), "layer tensors must be contiguous"
        self.struct = vl_lora_layer(T, d_in, d_out, r, int(w.F), int(w.eta),
                                    *[_ptr(getattr(w, n)) for n in LAYER_INT16 + LAYER_INT64])


def lora_chain_proof_size(layer: LayerArgs) -> int:
    return lib().vl_lora_chain_proof_size(ctypes.byref(layer.struct))


def lora_chain_workspace_size(layer: LayerArgs) -> int:
    return lib().vl_lora_chain_workspace_size(ctypes.byref(layer.struct))


def lora_chain_prove(layer: LayerArgs, seed: int, workspace=None, stream=None):
    """Blocking chained proof of one layer's step: returns (proof bytes,
    final transcript state)."""
    import torch
    if workspace is None:
        workspace = torch.empty(max(256, lora_chain_workspace_size(layer)), dtype=torch.uint8, device="cuda")
    n = lora_chain_proof_size(layer)
    buf = ctypes.create_string_buffer(max(n, 1))
    dig = ctypes.create_string_buffer(32)
    _check(lib().vl_lora_chain_prove(ctypes.byref(layer.struct), seed, workspace.data_ptr(),
                                     workspace.numel() * workspace.element_size(), ctypes.addressof(buf), n,
                                     ctypes.addressof(dig), _stream(stream)))
    return buf.raw[:n], dig.raw


def verify_transcript(proof: bytes, group: GroupArgs, seed: int):
    """Host verifier.  Returns (ok, fail_round, reduced claims as ints)."""
    cap = 4096
    red = (vl_fr * cap)()
    rlen = c_u64(0)
    fr_ = c_i32(0)
    buf = ctypes.create_string_buffer(proof, max(len(proof), 1))
    st = lib().vl_verify_transcript(ctypes.addressof(buf), len(proof), ctypes.byref(group.struct), seed,
                                    red, cap, ctypes.byref(rlen), ctypes.byref(fr_))
    if st not in (VL_OK, VL_ERR_REJECT):
        _check(st)
    return st == VL_OK, fr_.value, [fr_to_int(red[i]) for i in range(rlen.value)] if st == VL_OK else []


# ------------------------------------------------------- batched products --
class BmmArgs:
    """vl_bmm over H head matrices of each operand inside stored tensors
    (torch tensors on the device for proving, numpy arrays or None on the
    host for verification): head h of A starts head_stride_a elements after
    head h - 1, row-major with leading dimension lda (likewise B, C).  The
    tensors are kept alive as long as the structure is used."""

    def __init__(self, A, B, C, H: int, D0: int, D1: int, D2: int, lda: int, ldb: int, ldc: int,
                 head_stride_a: int, head_stride_b: int, head_stride_c: int, trans_a: bool = False,
                 trans_b: bool = False, group_id: int = 0, dtypes=None):
        self.keep = (A, B, C)
        dts = dtypes or [dtype_code(x.dtype) for x in (A, B, C)]
        ptr = lambda x: _ptr(x) if x is not None else None  # noqa: E731
        self.struct = vl_bmm(ptr(A), ptr(B), ptr(C), dts[0], dts[1], dts[2], H, D0, D1, D2, lda, ldb, ldc,
                             head_stride_a, head_stride_b, head_stride_c, int(bool(trans_a)), int(bool(trans_b)),
                             group_id)

    @property
    def dims(self):
        s = self.struct
        return (s.H, s.D0, s.D1, s.D2)


def bmm_proof_size(b: BmmArgs) -> int:
    return lib().vl_bmm_proof_size(ctypes.byref(b.struct))


def bmm_workspace_size(batches: Sequence[BmmArgs]) -> int:
    arr = (vl_bmm * len(batches))(*[b.struct for b in batches])
    return lib().vl_bmm_workspace_size(arr, len(batches))


def bmm_prove(batches: Sequence[BmmArgs], seed: int, workspace=None, stream=None):
    """Blocking proofs of batched products: returns (proofs, digests), one
    bytes object each per product."""
    import torch
    n = len(batches)
    arr = (vl_bmm * n)(*[b.struct for b in batches])
    if workspace is None:
        workspace = torch.empty(max(256, lib().vl_bmm_workspace_size(arr, n)), dtype=torch.uint8, device="cuda")
    total = sum(bmm_proof_size(b) for b in batches)
    buf = ctypes.create_string_buffer(max(total, 1))
    dig = ctypes.create_string_buffer(32 * n)
    offs = (c_u64 * (n + 1))()
    _check(lib().vl_bmm_prove(arr, n, seed, workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                              ctypes.addressof(buf), total, offs, ctypes.addressof(dig), _stream(stream)))
    raw = buf.raw
    return [raw[offs[k]:offs[k + 1]] for k in range(n)], [dig.raw[32 * k:32 * k + 32] for k in range(n)]


def bmm_verify(proof: bytes, b: BmmArgs, seed: int):
    """Host verifier of one batched proof.  Returns (ok, fail_round, reduced
    claims as ints)."""
    cap = 4096
    red = (vl_fr * cap)()
    rlen = c_u64(0)
    fr_ = c_i32(0)
    buf = ctypes.create_string_buffer(proof, max(len(proof), 1))
    st = lib().vl_bmm_verify(ctypes.addressof(buf), len(proof), ctypes.byref(b.struct), seed, red, cap,
                             ctypes.byref(rlen), ctypes.byref(fr_))
    if st not in (VL_OK, VL_ERR_REJECT):
        _check(st)
    return st == VL_OK, fr_.value, [fr_to_int(red[i]) for i in range(rlen.value)] if st == VL_OK else []


# --------------------------------------------------------------- lookups --
class LookupArgs:
    """vl_lookup over the entries x (and y) of a secret tensor and the table
    rows (t0 + j[, tb_j]) for j < N: torch tensors on the device for proving,
    numpy arrays (or None: shape only) on the host for verification.  With
    two_col the second columns y and tb are used."""

    def __init__(self, x, y, tb, t0: int, N: int, D: int, dtype, two_col: bool, lid: int = 0, dtype_y=None):
        self.keep = (x, y, tb)
        ptr = lambda v: _ptr(v) if v is not None else None  # noqa: E731
        dy = dtype_code(dtype_y) if dtype_y is not None else 0
        self.struct = vl_lookup(ptr(x), ptr(y), ptr(tb), dtype_code(dtype), dy, t0, int(bool(two_col)), N, D, lid)


def lookup_proof_size(a: LookupArgs) -> int:
    return lib().vl_lookup_proof_size(ctypes.byref(a.struct))


def lookup_workspace_size(args: Sequence[LookupArgs]) -> int:
    arr = (vl_lookup * len(args))(*[a.struct for a in args])
    return lib().vl_lookup_workspace_size(arr, len(args))


def lookup_prove(args: Sequence[LookupArgs], seed: int, workspace=None, stream=None):
    """Blocking lookup proofs: returns (proofs, digests)."""
    import torch
    n = len(args)
    arr = (vl_lookup * n)(*[a.struct for a in args])
    if workspace is None:
        workspace = torch.empty(max(256, lib().vl_lookup_workspace_size(arr, n)), dtype=torch.uint8, device="cuda")
    total = sum(lookup_proof_size(a) for a in args)
    buf = ctypes.create_string_buffer(max(total, 1))
    dig = ctypes.create_string_buffer(32 * n)
    offs = (c_u64 * (n + 1))()
    _check(lib().vl_lookup_prove(arr, n, seed, workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                                 ctypes.addressof(buf), total, offs, ctypes.addressof(dig), _stream(stream)))
    raw = buf.raw
    return [raw[offs[k]:offs[k + 1]] for k in range(n)], [dig.raw[32 * k:32 * k + 32] for k in range(n)]


def lookup_verify(proof: bytes, a: LookupArgs, seed: int):
    """Host verifier of one lookup proof: (ok, fail_round, reduced)."""
    cap = 4096
    red = (vl_fr * cap)()
    rlen = c_u64(0)
    fr_ = c_i32(0)
    buf = ctypes.create_string_buffer(proof, max(len(proof), 1))
    st = lib().vl_lookup_verify(ctypes.addressof(buf), len(proof), ctypes.byref(a.struct), seed, red, cap,
                                ctypes.byref(rlen), ctypes.byref(fr_))
    if st not in (VL_OK, VL_ERR_REJECT):
        _check(st)
    return st == VL_OK, fr_.value, [fr_to_int(red[i]) for i in range(rlen.value)] if st == VL_OK else []


# ---------------------------------------------------------------- Hyrax ------
HYRAX_POINT_BYTES = 96


def hyrax_windows(dtype) -> int:
    """Table windows an entry type needs: its size in bytes."""
    return {VL_I16: 2, VL_I32: 4, VL_I64: 8}[dtype_code(dtype)]


def hyrax_table_size(m: int, windows: int) -> int:
    return lib().vl_hyrax_table_size(m, windows)


class HyraxTable:
    """Device fixed-base table (public parameters) of m generators and the
    given windows, filled by vl_hyrax_setup on the current stream."""

    def __init__(self, m: int, windows: int = 2, stream=None):
        import torch
        self.m, self.windows = m, windows
        n = hyrax_table_size(m, windows)
        if n == 0:
            raise VLError(VL_ERR_SHAPE, "bad Hyrax table shape")
        self.buf = torch.empty(n, dtype=torch.uint8, device="cuda")
        _check(lib().vl_hyrax_setup(m, windows, self.buf.data_ptr(), n, _stream(stream)))


def hyrax_commit_workspace_size(R: int, m: int, split: int = 0) -> int:
    return lib().vl_hyrax_commit_workspace_size(R, m, split)


def hyrax_commit(M, table: HyraxTable, out=None, workspace=None, split: int = 0, stream=None):
    """Row commitments of the device matrix M (R x m int16/int32/int64) as a
    device uint8 tensor of R x 96 bytes (asynchronous on the stream)."""
    import torch
    R, m = M.shape
    if out is None:
        out = torch.empty((R, HYRAX_POINT_BYTES), dtype=torch.uint8, device=M.device)
    need = hyrax_commit_workspace_size(R, m, split)
    if workspace is None:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=M.device)
    _check(lib().vl_hyrax_commit(_ptr(M), dtype_code(M.dtype), R, m, _row_stride(M), table.buf.data_ptr(), table.m,
                                 table.windows, split, _ptr(out), _ptr(workspace),
                                 workspace.numel() * workspace.element_size(), _stream(stream)))
    return out


def hyrax_generators(m: int) -> bytes:
    """The generators G_0 .. G_{m-1} computed on the host (96 bytes each)."""
    buf = ctypes.create_string_buffer(HYRAX_POINT_BYTES * m)
    _check(lib().vl_hyrax_generators(m, ctypes.addressof(buf)))
    return buf.raw


def hyrax_open(M, x: Sequence[int], stream=None) -> List[int]:
    """The opening message w = sum_i eq(x, i) M[i][.] of a device matrix,
    computed by the device partial evaluation (eq table, VL_CONTRACT_ROWS,
    export to canonical form); returns the m canonical values."""
    import torch
    R, m = M.shape
    n_eq = 1 << len(x)
    eq = torch.empty((8, max(n_eq, R)), dtype=torch.int32, device=M.device)
    eq_table(x, fr_vec(eq, n_eq), stream)
    out = torch.empty((8, m), dtype=torch.int32, device=M.device)
    ws_n = partial_eval_workspace_size(R, m, VL_CONTRACT_ROWS, M.dtype)
    ws = torch.empty(max(ws_n, 256), dtype=torch.uint8, device=M.device)
    mle_partial_eval(M, VL_CONTRACT_ROWS, fr_vec(eq, max(n_eq, R)), fr_vec(out), ws, stream)
    canon = torch.empty((m, 8), dtype=torch.int32, device=M.device)
    fr_export(fr_vec(out), m, canon, stream)
    torch.cuda.synchronize()
    words = canon.cpu().numpy().astype("uint32")
    return [sum(int(words[j, k]) << (32 * k) for k in range(8)) for j in range(m)]


def hyrax_verify_open(commits: bytes, R: int, m: int, x: Sequence[int], y: Sequence[int], w: Sequence[int]):
    """Host check of an opening: (ok, value, message)."""
    xa = (vl_fr * max(1, len(x)))(*[int_to_fr(v) for v in x])
    ya = (vl_fr * max(1, len(y)))(*[int_to_fr(v) for v in y])
    wa = (vl_fr * max(1, len(w)))(*[int_to_fr(v) for v in w])
    val = vl_fr()
    buf = ctypes.create_string_buffer(bytes(commits), max(len(commits), 1))
    st = lib().vl_hyrax_verify_open(ctypes.addressof(buf), R, m, xa, ya, wa, ctypes.byref(val))
    if st not in (VL_OK, VL_ERR_REJECT):
        _check(st)
    return st == VL_OK, (fr_to_int(val) if st == VL_OK else None), ("" if st == VL_OK else last_error())
