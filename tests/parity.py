"""Shared helpers of the parity tests: error measures and cached synthetic cases.

Error measures (FP32 GPU result against the FP64 oracle on identical inputs):
  volume:   max |I - I_ref| / max |I_ref|                       (<= 1e-4)
  gradient: per parameter type k (tx..rz), max_j |g_jk - ref_jk| / max_j |ref_jk|  (<= 1e-3)
Normwise measures, because ramp-filtered data cross zero everywhere (pointwise
ratios are meaningless there) and translations and rotations differ in scale.
"""
from __future__ import annotations

import functools

import numpy as np

VOL_TOL = 1e-4
GRAD_TOL = 1e-3


def vol_err(got, ref) -> float:
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def grad_err(got, ref) -> np.ndarray:
    got = np.asarray(got, dtype=np.float64).reshape(-1, 6)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1, 6)
    return np.max(np.abs(got - ref), axis=0) / np.max(np.abs(ref), axis=0)


def mat_err(got, ref) -> float:
    """dL/dPhat: per view, max entry error over max entry magnitude, worst view."""
    got = np.asarray(got, dtype=np.float64).reshape(-1, 12)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1, 12)
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


@functools.lru_cache(maxsize=4)
def case(name: str, with_motion: bool = True):
    from synth import make_case

    return make_case(name, with_motion=with_motion)
