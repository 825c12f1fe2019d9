"""Marshal a workloads.LookupCase into the library's vl_lookup (test helper)."""
from paper_2508_21393_amd import binding as B


def lookup_args(lc, where: str = "host", to_device=None) -> "B.LookupArgs":
    """where = "host": numpy arrays (verification); "none": shape only;
    "device": to_device(numpy array) gives the device tensor."""
    two = lc.y is not None
    arrs = (lc.x, lc.y, lc.tb)
    if where == "none":
        ts = (None, None, None)
    elif where == "device":
        ts = tuple(to_device(a) if a is not None else None for a in arrs)
    else:
        ts = arrs
    return B.LookupArgs(ts[0], ts[1], ts[2], lc.t0, lc.N, len(lc.x), lc.x.dtype, two, lc.lid,
                        dtype_y=lc.y.dtype if two else None)
