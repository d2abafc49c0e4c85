"""Helpers for the GPU parity tests: device transfer and error norms."""
import os

import numpy as np


def ensure_lib():
    from paper_2109_06743_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()


def dev(a, dtype):
    import torch
    tdt = {"f32": torch.float32, "f64": torch.float64}.get(dtype, dtype)
    return torch.as_tensor(np.ascontiguousarray(a)).to(tdt).reshape(-1).contiguous().cuda()


def host(t, shape=None):
    a = t.detach().double().cpu().numpy()
    return a.reshape(shape) if shape is not None else a


def storage_round(a, dtype):
    """The values the device holds for `a` in storage type dtype, as FP64."""
    return np.asarray(a, dtype=np.float32 if dtype == "f32" else np.float64).astype(np.float64)


def rel_l2(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


# per-call tolerances on rel-L2(f): FP32 storage/arithmetic vs the FP64 oracle,
# and the FP64 path vs the oracle (rounding order only)
TOL_SWEEP = {"f32": 1e-6, "f64": 1e-13}
TOL_STEP = {"f32": 1e-5, "f64": 1e-12}
TOL_MOM = {"f32": 1e-6, "f64": 1e-12}
