"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module draws random numbers and evaluates closed-form input functions
(continuous Maxwellian mixtures) at velocity-grid nodes.  It holds none of the
solver's arithmetic: no discrete Maxwellian, no collision operator, no cell
solve.  Both the HIP path and the CPU oracle take its arrays as plain inputs.

Every generator takes an explicit integer seed; the stream for item ``i`` of a
batch is ``numpy.random.default_rng([seed, i])`` so that any single item can be
regenerated on its own (used for sampled parity checks at full size).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "grid_nodes",
    "maxwellian_mixture",
    "mixture_batch",
    "mixture_params",
    "cell_inflow_batch",
    "RH_states",
]


def grid_nodes(N: int, L: float) -> np.ndarray:
    """Per-axis node coordinates k*dv, k = -N/2+1 .. N/2, dv = 2L/N
    (Section 2.2, velocity discretization for the quadratic operator)."""
    dv = 2.0 * L / N
    return (np.arange(N, dtype=np.float64) - N // 2 + 1) * dv


def maxwellian_mixture(params, N: int, L: float, d: int = 3) -> np.ndarray:
    """Evaluate sum_i rho_i (2 pi T_i)^{-d/2} exp(-|v-u_i|^2 / 2T_i) at the
    grid nodes; returns a C-ordered array of shape (N,)*d flattened to N^d.
    ``params`` is a list of (rho, u[d], T)."""
    x = grid_nodes(N, L)
    f = np.zeros((N,) * d)
    for rho, u, T in params:
        # each component factorises over the axes
        comp = rho * (2.0 * np.pi * T) ** (-d / 2.0)
        fac = [np.exp(-((x - u[a]) ** 2) / (2.0 * T)) for a in range(d)]
        prod = fac[0]
        for a in range(1, d):
            prod = np.multiply.outer(prod, fac[a])
        f += comp * prod
    return f.reshape(-1)


def mixture_params(rng, d=3, n_range=(2, 4), rho=(0.5, 2.0), speed=(0.0, 1.5), T=(0.5, 2.0)):
    """Draw one cell's Maxwellian-mixture parameters: n ~ U{n_range}, each
    component rho ~ U(rho), |u| ~ U(speed) along a normalised standard normal
    direction, T ~ U(T)."""
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    out = []
    for _ in range(n):
        r = float(rng.uniform(*rho))
        direction = rng.standard_normal(d)
        direction /= np.linalg.norm(direction)
        u = direction * float(rng.uniform(*speed))
        t = float(rng.uniform(*T))
        out.append((r, u, t))
    return out


def mixture_batch(B: int, N: int, L: float, d: int = 3, seed: int = 0, start: int = 0, **kw) -> np.ndarray:
    """Batch of B cells [B, N^d] (float64); cell i uses rng([seed, start+i])."""
    out = np.empty((B, N ** d))
    for i in range(B):
        rng = np.random.default_rng([seed, start + i])
        out[i] = maxwellian_mixture(mixture_params(rng, d=d, **kw), N, L, d)
    return out


def cell_inflow_batch(B: int, N: int, L: float, dx: float, d: int = 3, seed: int = 1, start: int = 0):
    """Upwind-neighbour data for independent cell solves.  Returns
    (f_old, f_left, f_right, eps) where f_old, f_left, f_right are Maxwellian
    mixtures [B, N^d] and eps[B] is log-uniform in [0.005, 1].  The caller
    forms the transport right-hand side from the neighbours."""
    f_old = np.empty((B, N ** d))
    f_left = np.empty((B, N ** d))
    f_right = np.empty((B, N ** d))
    eps = np.empty(B)
    for i in range(B):
        rng = np.random.default_rng([seed, start + i])
        f_old[i] = maxwellian_mixture(mixture_params(rng, d=d, speed=(0.0, 0.5), T=(0.8, 1.5)), N, L, d)
        f_left[i] = maxwellian_mixture(mixture_params(rng, d=d, speed=(0.0, 0.5), T=(0.8, 1.5)), N, L, d)
        f_right[i] = maxwellian_mixture(mixture_params(rng, d=d, speed=(0.0, 0.5), T=(0.8, 1.5)), N, L, d)
        eps[i] = float(np.exp(rng.uniform(np.log(0.005), np.log(1.0))))
    return f_old, f_left, f_right, eps


def RH_states(mach: float, gas_gamma: float = 5.0 / 3.0):
    """Upstream/downstream states of a monatomic normal shock with p = rho T,
    upstream rho=1, T=1 (Rankine-Hugoniot jump relations).  Returns
    ((rho1, u1, T1), (rho2, u2, T2))."""
    g = gas_gamma
    m2 = mach * mach
    rho_ratio = (g + 1.0) * m2 / ((g - 1.0) * m2 + 2.0)
    T_ratio = (2.0 * g * m2 - (g - 1.0)) * ((g - 1.0) * m2 + 2.0) / ((g + 1.0) ** 2 * m2)
    u1 = mach * np.sqrt(g)
    return (1.0, u1, 1.0), (rho_ratio, u1 / rho_ratio, T_ratio)
