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


def _maxw_grid(rho, u0, T, N, L, d=3, v1_shift=0.0):
    """rho M(u0 e_1, T) at the nodes of a grid whose axis 0 is shifted by v1_shift."""
    x = grid_nodes(N, L)
    fac = [np.exp(-((x + (v1_shift if a == 0 else 0.0) - (u0 if a == 0 else 0.0)) ** 2) / (2.0 * T))
           for a in range(d)]
    prod = fac[0]
    for a in range(1, d):
        prod = np.multiply.outer(prod, fac[a])
    return (rho * (2.0 * np.pi * T) ** (-d / 2.0) * prod).reshape(-1)


def warmstart_cells(n_inst: int, cells_per_inst: int, N: int, L: float, seed: int = 7, start: int = 0):
    """Cell states of the two families used to train and test the learned warm
    start: normal-shock profiles (Mach ~ U(2, 4), Rankine-Hugoniot end states,
    velocities centred on the mean of the two bulk speeds, a smooth blend of
    the two Maxwellians across a width delta ~ U(0.5, 2)) for even instance
    indices, and heat-slab profiles (T_L = 1, T_R ~ U(1.5, 2.5), rho ~ 1/T, a
    heat-flux perturbation of amplitude ~ eps) for odd ones.  eps is
    log-uniform in [0.005, 1] per instance.  Returns (f_left, f_old, f_right,
    eps) with shapes [n_inst * cells_per_inst, N^3] and [n_inst * cells_per_inst]."""
    K = N ** 3
    n = n_inst * cells_per_inst
    fl, fo, fr = np.empty((n, K)), np.empty((n, K)), np.empty((n, K))
    eps = np.empty(n)
    x = grid_nodes(N, L)
    v1 = np.repeat(x, N * N)
    v2 = (np.add.outer(np.add.outer(x * x, x * x), x * x)).reshape(-1)
    for i in range(n_inst):
        rng = np.random.default_rng([seed, start + i])
        e = float(np.exp(rng.uniform(np.log(0.005), np.log(1.0))))
        if (start + i) % 2 == 0:
            mach = float(rng.uniform(2.0, 4.0))
            (r1, u1, T1), (r2, u2, T2) = RH_states(mach)
            ub = 0.5 * (u1 + u2)
            delta = float(rng.uniform(0.5, 2.0))
            M1 = _maxw_grid(r1, u1 - ub, T1, N, L)
            M2 = _maxw_grid(r2, u2 - ub, T2, N, L)
            h = delta / 4.0
            for c in range(cells_per_inst):
                xc = float(rng.uniform(-3.0 * delta, 3.0 * delta))
                for arr, xx in ((fl, xc - h), (fo, xc), (fr, xc + h)):
                    wgt = 1.0 / (1.0 + np.exp(-xx / delta))
                    arr[i * cells_per_inst + c] = (1.0 - wgt) * M1 + wgt * M2
        else:
            TR = float(rng.uniform(1.5, 2.5))
            a = min(e, 0.3) * (TR - 1.0) * 0.5
            for c in range(cells_per_inst):
                xc = float(rng.uniform(0.05, 0.95))
                for arr, xx in ((fl, xc - 1.0 / 32), (fo, xc), (fr, xc + 1.0 / 32)):
                    T = 1.0 + (TR - 1.0) * xx
                    M = _maxw_grid(1.0 / T, 0.0, T, N, L)
                    pert = 1.0 + a * (v1 / np.sqrt(T)) * (v2 / (2.0 * T) - 2.5)
                    arr[i * cells_per_inst + c] = np.maximum(M * pert, 0.0)
        eps[i * cells_per_inst:(i + 1) * cells_per_inst] = e
    return fl, fo, fr, eps


def shock_step(mach: float, nx: int, N: int, L: float, xL: float = -20.0, xR: float = 20.0, v1_shift: float = 0.0):
    """Initial state of the normal-shock problem: the upstream Rankine-Hugoniot
    Maxwellian in the cells left of x = 0 and the downstream one right of it, on
    a velocity grid whose axis 0 is shifted by v1_shift.  Returns (f [nx, N^3],
    upstream (rho, u, T), downstream (rho, u, T))."""
    up, down = RH_states(mach)
    dx = (xR - xL) / nx
    xc = xL + (np.arange(nx) + 0.5) * dx
    fu = _maxw_grid(up[0], up[1], up[2], N, L, v1_shift=v1_shift)
    fd = _maxw_grid(down[0], down[1], down[2], N, L, v1_shift=v1_shift)
    f = np.where((xc < 0.0)[:, None], fu[None, :], fd[None, :])
    return np.ascontiguousarray(f), up, down


def shock_instances(n: int = 16, mach=(2.0, 4.0), eps_cycle=(1.0, 0.1, 0.01)):
    """Batched shock workload: Mach numbers linspace(mach), eps cycling through eps_cycle."""
    machs = np.linspace(mach[0], mach[1], n)
    return [(float(machs[i]), float(eps_cycle[i % len(eps_cycle)])) for i in range(n)]
