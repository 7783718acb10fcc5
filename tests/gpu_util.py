"""Shared helpers of the GPU tests (not collected: no test_ prefix)."""
from __future__ import annotations

import sys

import numpy as np


def announce(msg):
    """Name the GPU case before it runs (so a failure that ends the process is attributable)."""
    sys.stdout.write(f"\n[gpu-case] {msg}\n")
    sys.stdout.flush()


def fp_error(f_gpu, f_ref, mask, dtype):
    """max abs error (f64) or max relative error (other dtypes) over fluid slots."""
    fl = mask == 0
    a = f_gpu[:, fl]
    b = f_ref[:, fl]
    if dtype == "f64":
        return float(np.abs(a - b).max()) if a.size else 0.0
    return float((np.abs(a - b) / np.abs(b)).max()) if a.size else 0.0


TOL = {"f64": 1e-12, "f32": 1e-5}
