"""Shared helpers of the GPU tests (inputs and comparisons only)."""
import sys

import numpy as np
import torch


# Bars on the relative Frobenius error of sigma against the oracle's FP64
# sigma.  FP64 and FP32: the stated tolerances.  BF16x3: every operand x is
# carried as hi + lo (two BF16 roundings to nearest even, 8-bit
# significands, u = 2^-8), leaving |x - hi - lo| <= u^2 |x|, about u^2 / 3 in
# root mean square; each product drops lo*lo (rms about u^2 / 3 as well).
# A task goes through two such products (phase A: X and M split, lo*lo
# dropped; phase B: T and Y split, lo*lo dropped) plus the FP32 rounding of
# the inputs (2^-24), six independent sources of rms u^2 / 3: about
# sqrt(6) 2^-16 / 3 = 1.2e-5 relative per task term.  Sums over terms and
# over the inner dimensions average such errors, so the relative error of
# sigma stays at or below that (3.7e-6 measured on the D = 4096 workload);
# the bar is 2e-5, 1.6x the estimate.
SIGMA_TOL = {"f64": 1e-12, "f32": 1e-6, "bf16x3": 2e-5}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype=dtype)
