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

# Lattice weights w_i (Eq. 6), the natural scale of population i.
_W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def fp_error_w(f_gpu, f_ref, mask, dtype):
    """As fp_error, but FP32 errors are taken relative to max(|f_ref|, w_i): flows with open
    boundaries drive some populations far below their weight (next to a moving lid's corners
    f_7 falls to 1e-4 against w_7 = 1/36), where the error of the 32-bit deviation storage
    stays at its absolute level (a few 1e-9) while the value-relative error loses meaning."""
    fl = mask == 0
    a = f_gpu[:, fl]
    b = f_ref[:, fl]
    if not a.size:
        return 0.0
    if dtype == "f64":
        return float(np.abs(a - b).max())
    return float((np.abs(a - b) / np.maximum(np.abs(b), _W[:, None])).max())
