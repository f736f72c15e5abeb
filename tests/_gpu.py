"""Helpers shared by the GPU parity tests (compare the HIP path with the CPU
oracle on the same seeded inputs)."""
import numpy as np

import oracle

U = np.finfo(np.float64).eps / 2


def torch_dev():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need an MI355X; run them with -m gpu on the GPU box")
    return torch


def d4_tol(sigma: float) -> float:
    """Relative (per column, infinity norm) parity tolerance for I + sigma*D4.
    Both sides are backward stable banded LU solves of an SPD matrix, so
    they may differ by a few units of rounding times kappa_2 <= 1 + 16 sigma;
    64 u (1 + 16 sigma) leaves room for the different rounding order (stored
    reciprocals, fused multiply-adds, the segment decomposition)."""
    return 64 * U * (1 + 16 * sigma)


def colerr(X, ref):
    """max_i |X_ij - ref_ij| / max_i |ref_ij|, per column."""
    num = np.max(np.abs(X - ref), axis=0)
    den = np.maximum(np.max(np.abs(ref), axis=0), 1e-300)
    return num / den


def print_case(**kw):
    print("CASE " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)
