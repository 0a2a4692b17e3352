"""Helpers of the GPU tests: device buffers and calls through the C ABI."""
import sys

import numpy as np


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a visible GPU")
    return torch.device("cuda:0")


def to_dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x).reshape(-1)).to(dev())


def run_correlate(cpi, fa, fb, n, pa, pb, fmt, layout, outputs=("gamma", "gamma_f32", "numer"),
                  sums=True):
    """Runs cpi_correlate on host frame arrays; returns host copies of every output."""
    import torch

    d = dev()
    da, db = to_dev(fa), to_dev(fb)
    res = {}
    kw = {}
    if "gamma" in outputs:
        kw["gamma"] = torch.full((pa * pb,), np.nan, dtype=torch.float64, device=d)
    if "gamma_f32" in outputs:
        kw["gamma_f32"] = torch.full((pa * pb,), np.nan, dtype=torch.float32, device=d)
    if "numer" in outputs:
        kw["numer"] = torch.full((pa * pb,), -7, dtype=torch.int64, device=d)
    if sums:
        kw["sum_a"] = torch.full((pa,), -7, dtype=torch.int64, device=d)
        kw["sum_b"] = torch.full((pb,), -7, dtype=torch.int64, device=d)
    cpi.correlate(da, db, n, pa, pb, fmt, layout, **kw)
    torch.cuda.synchronize()
    for k, v in kw.items():
        res[k] = v.cpu().numpy()
    return res


def oracle_in_layout(ref, layout):
    import oracle

    return {
        "gamma": oracle.to_layout(ref["gamma"], layout).reshape(-1),
        "gamma_f32": oracle.to_layout(ref["gamma_f32"], layout).reshape(-1),
        "numer": oracle.to_layout(ref["numer"], layout).reshape(-1),
        "sum_a": ref["sum_a"],
        "sum_b": ref["sum_b"],
    }


def assert_bit_exact(got, want, what=""):
    for k in got:
        g, w = got[k], want[k]
        if g.dtype.kind == "f":
            ok = np.array_equal(g.view(np.uint64 if g.itemsize == 8 else np.uint32),
                                np.ascontiguousarray(w, dtype=g.dtype).view(
                                    np.uint64 if g.itemsize == 8 else np.uint32))
        else:
            ok = np.array_equal(g, w)
        if not ok:
            bad = np.flatnonzero(g != np.asarray(w, dtype=g.dtype))
            raise AssertionError(f"{what}{k}: {bad.size} mismatches, first at {bad[:5]}: "
                                 f"got {g[bad[:5]]}, want {np.asarray(w)[bad[:5]]}")


def plane_rel_err(got, want):
    """Per-plane max-abs error over max-abs value (the refocus tolerance)."""
    got = np.asarray(got, dtype=np.float64).reshape(want.shape[0], -1)
    want = np.asarray(want, dtype=np.float64).reshape(want.shape[0], -1)
    scale = np.abs(want).max(axis=1)
    scale[scale == 0] = 1.0
    return np.abs(got - want).max(axis=1) / scale
