"""Marshal a workloads.HeadBatch into the library's vl_bmm (test helper)."""
from paper_2508_21393_amd import binding as B


def bmm_args(hb, where: str = "host", to_device=None) -> "B.BmmArgs":
    """where = "host": the stored numpy arrays (verification); "none": shape
    only; "device": to_device(numpy array) gives the device tensor."""
    H, D0, D1, D2 = hb.dims
    arrs = (hb.A.base, hb.B.base, hb.C.base)
    dts = [B.dtype_code(a.dtype) for a in arrs]
    if where == "none":
        ts = (None, None, None)
    elif where == "device":
        ts = tuple(to_device(a) for a in arrs)
    else:
        ts = arrs
    return B.BmmArgs(ts[0], ts[1], ts[2], H, D0, D1, D2, hb.A.ld, hb.B.ld, hb.C.ld, hb.A.head_stride,
                     hb.B.head_stride, hb.C.head_stride, hb.transA, hb.transB, hb.group_id, dtypes=dts)
