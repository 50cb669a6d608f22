"""Helpers shared by the GPU parity tests (device transfers, error norms).

With YEEPIC_ERRLOG set to a file path, every checked error is appended to it
as one JSON line (test, quantity, error, tolerance), so that the measured
error of each result can be stated next to its bound."""
import json
import os

import numpy as np
import torch

DEV = "cuda:0"


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype).contiguous()


def host(t):
    return t.detach().to("cpu", torch.float64).numpy()


def fields_dev(E, B, dtype=torch.float64):
    return [dev(e, dtype) for e in E], [dev(x, dtype) for x in B]


def record(what, err, tol):
    """Append a measured error to the YEEPIC_ERRLOG file (if set)."""
    path = os.environ.get("YEEPIC_ERRLOG")
    if not path:
        return
    test = os.environ.get("PYTEST_CURRENT_TEST", "").split(" ")[0]
    with open(path, "a") as f:
        f.write(json.dumps({"test": test, "what": what, "err": float(err), "tol": float(tol)}) + "\n")


def check(err, tol, what):
    """Record ``err`` and assert err <= tol."""
    record(what, err, tol)
    assert err <= tol, f"{what}: error {err:.3e} > {tol:.1e}"


def normwise(got, ref):
    """max|got - ref| / max|ref| (one field component)."""
    scale = np.max(np.abs(ref))
    return float(np.max(np.abs(got - ref)) / (scale if scale > 0 else 1.0))


def assert_fields_close(got, ref, tol, what="", joint=False):
    """Per component max|got - ref| <= tol * scale, with scale = max|ref| of
    that component, or (joint) of the largest component of the same field.
    Joint is for fields whose components differ by orders of magnitude (a
    laser with the plasma's response): every component then carries the
    rounding of the strong ones (ulps of max|E| through the curl), in FP64 as
    in FP32, so a per-component bound would measure the float format; the
    per-component errors are still recorded (tolerance inf)."""
    joint_scale = max(float(np.max(np.abs(r))) for r in ref) if joint else None
    for c, (g, r) in enumerate(zip(got, ref)):
        gh = host(g) if isinstance(g, torch.Tensor) else g
        if joint:
            err = float(np.max(np.abs(gh - r))) / (joint_scale if joint_scale > 0 else 1.0)
            record(f"{what} component {c + 1} (own scale)", normwise(gh, r), float("inf"))
        else:
            err = normwise(gh, r)
        record(f"{what} component {c + 1}", err, tol)
        assert err <= tol, f"{what} component {c + 1}: norm-wise error {err:.3e} > {tol:.1e}"
