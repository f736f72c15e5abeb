"""Seeded synthetic inputs for the batched pentadiagonal workloads.

This module only draws numbers (numpy PCG64, one stream per seed); it holds
none of the solver's arithmetic, so both the HIP path and the CPU oracle can
consume exactly the same bits.  Every array is returned in the interleaved,
batch-fastest layout (shape (n, systems), row i = unknown i of every system).

Workloads (all synthetic; the paper benchmarks batches of synthetic
hyperdiffusion runs, Sec. 3):

* ``plain``      : N=256, sigma=0.1, 256 right-hand sides uniform[-1, 1).
* ``hyperdiff``  : N=4096, sigma=50, 65536 systems, C^0 uniform[-1, 1),
                   100 backward-Euler steps.
* ``cahn2d``     : 1024 x 1024 grid, 32 instances, sigma=200,
                   gamma_k = 10**U(-3, -1), C^0 uniform[-0.1, 0.1), 50 steps.
* ``precision``  : N=8192, 131072 right-hand sides uniform[-1, 1) rounded once
                   to FP32, sigma in {1, 1e2, 1e4}.
* ``group``      : 48 matrices, sigma_k = 10**U(-2, 4),
                   N_k = round(exp(U(ln 64, ln 8192))),
                   R_k = round(exp(U(ln 8, ln 8192))), entries uniform[-1, 1),
                   200 backward-Euler steps.
"""
from __future__ import annotations

import math

import numpy as np

PLAIN = dict(n=256, sigma=0.1, batch=256, seed=1)
HYPERDIFF = dict(n=4096, sigma=50.0, batch=65536, steps=100, seed=2)
CAHN2D = dict(nx=1024, ninst=32, sigma=200.0, steps=50, seed=3)
PRECISION = dict(n=8192, batch=131072, sigmas=(1.0, 1e2, 1e4), seed=4)
GROUP = dict(count=48, steps=200, seed=5)
PERIODIC = dict(n=4096, sigma=50.0, batch=65536, steps=250, seed=6)
REWRITE = dict(n=1024, batch=65536, seed=7)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform(seed: int, shape, lo: float = -1.0, hi: float = 1.0,
            row_block: int = 256) -> np.ndarray:
    """uniform[lo, hi) FP64 of the given 2-D shape, drawn row block by row
    block from one stream (identical to a single draw of the whole array,
    but with a bounded temporary)."""
    g = rng(seed)
    out = np.empty(shape, dtype=np.float64)
    n = shape[0]
    for r0 in range(0, n, row_block):
        r1 = min(n, r0 + row_block)
        out[r0:r1] = g.uniform(lo, hi, size=(r1 - r0,) + tuple(shape[1:]))
    return out


def plain(seed: int = PLAIN["seed"], n: int = PLAIN["n"], batch: int = PLAIN["batch"]):
    return dict(n=n, sigma=PLAIN["sigma"], F=uniform(seed, (n, batch)))


def hyperdiff(seed: int = HYPERDIFF["seed"], n: int = HYPERDIFF["n"],
              batch: int = HYPERDIFF["batch"]):
    return dict(n=n, sigma=HYPERDIFF["sigma"], C0=uniform(seed, (n, batch)))


def periodic(seed: int = PERIODIC["seed"], n: int = PERIODIC["n"],
             batch: int = PERIODIC["batch"]):
    """Periodic Crank-Nicolson hyperdiffusion batch: C^0 uniform[-1, 1) per
    system (the step matrix is the same for every system)."""
    return dict(n=n, sigma=PERIODIC["sigma"], C0=uniform(seed, (n, batch)))


def rewrite(seed: int = REWRITE["seed"], n: int = REWRITE["n"], batch: int = REWRITE["batch"]):
    """A matrix per system: sigma_j = 10^U(-2, 4) (system j = I + sigma_j D4),
    right-hand sides uniform[-1, 1)."""
    g = rng(seed)
    return dict(n=n, sigma=10.0 ** g.uniform(-2.0, 4.0, size=batch), F=uniform(seed + 1000, (n, batch)))


def cahn2d(seed: int = CAHN2D["seed"], nx: int = CAHN2D["nx"], ninst: int = CAHN2D["ninst"]):
    """gamma per instance and C^0 of shape (ny, ninst, nx) = [y][inst][x]."""
    g = rng(seed)
    gammas = 10.0 ** g.uniform(-3.0, -1.0, size=ninst)
    C0 = uniform(seed + 1000, (nx, ninst * nx), -0.1, 0.1).reshape(nx, ninst, nx)
    return dict(nx=nx, ninst=ninst, sigma=CAHN2D["sigma"], gammas=gammas, C0=C0)


def precision(seed: int = PRECISION["seed"], n: int = PRECISION["n"],
              batch: int = PRECISION["batch"]):
    """FP64 uniform[-1, 1) draws rounded once (to nearest even) to FP32."""
    F64 = uniform(seed, (n, batch))
    return dict(n=n, F32=F64.astype(np.float32))


def group_shapes(seed: int = GROUP["seed"], count: int = GROUP["count"]):
    """(sigma_k, N_k, R_k) for the many-matrix workload."""
    g = rng(seed)
    sig = 10.0 ** g.uniform(-2.0, 4.0, size=count)
    ns = np.rint(np.exp(g.uniform(math.log(64), math.log(8192), size=count))).astype(np.int64)
    rs = np.rint(np.exp(g.uniform(math.log(8), math.log(8192), size=count))).astype(np.int64)
    return [(float(s), int(n), int(r)) for s, n, r in zip(sig, ns, rs)]


def group(seed: int = GROUP["seed"], count: int = GROUP["count"], max_cols: int | None = None):
    """List of (sigma_k, F_k) with F_k uniform[-1, 1) of shape (N_k, R_k).
    ``max_cols`` keeps only the first columns of every block (same values)."""
    out = []
    for k, (s, n, r) in enumerate(group_shapes(seed, count)):
        F = uniform(seed * 1000 + k, (n, r))
        if max_cols is not None:
            F = np.ascontiguousarray(F[:, :max_cols])
        out.append((s, F))
    return out
