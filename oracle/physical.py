"""Direct physical-space quadrature of the collision integral (oracle; test
infrastructure only).

eq. collision in its sigma-representation, with v_* = v - g, g = rho ghat,
v' = v - g/2 + rho sigma/2, v'_* = v - g/2 - rho sigma/2, kernel B = |g|^gamma
and the relative speed truncated at R_g (the truncation the spectral method
uses, Section 4.2):
  Q+(v) = int_0^{R_g} rho^{gamma+d-1} int_S int_S f(v') f(v'_*) dsigma dghat drho
  Q-(v) = f(v) |S^{d-1}| int_0^{R_g} rho^{gamma+d-1} int_S f(v - rho ghat) dghat drho.
f is an analytic Maxwellian mixture evaluated directly (not on a grid), so this
shares nothing with the Fourier machinery and pins its derivation: factors of
1/2 in the shifts, the rho^{d-1} measure, the S_d factors and signs.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial.legendre import leggauss


def _sphere(d: int, n: int):
    if d == 3:
        c, wc = leggauss(n)
        ph = 2.0 * np.pi * (np.arange(2 * n) + 0.5) / (2 * n)
        C, P = np.meshgrid(c, ph, indexing="ij")
        S = np.sqrt(1.0 - C * C)
        pts = np.stack([C.ravel(), (S * np.cos(P)).ravel(), (S * np.sin(P)).ravel()], axis=1)
        w = np.repeat(wc, 2 * n) * (2.0 * np.pi / (2 * n))
        return pts, w
    th = 2.0 * np.pi * (np.arange(n) + 0.5) / n
    return np.stack([np.cos(th), np.sin(th)], axis=1), np.full(n, 2.0 * np.pi / n)


def mixture_eval(params, x: np.ndarray) -> np.ndarray:
    """Continuous Maxwellian mixture at points x[..., d]."""
    d = x.shape[-1]
    out = np.zeros(x.shape[:-1])
    for rho, u, T in params:
        r2 = ((x - np.asarray(u)) ** 2).sum(-1)
        out += rho * (2.0 * np.pi * T) ** (-d / 2.0) * np.exp(-r2 / (2.0 * T))
    return out


def q_physical(params, v: np.ndarray, d: int, R_g: float, gamma: float = 0.0,
               n_rho: int = 40, n_sph: int = 16):
    """(gain, loss) at each point of v[P, d] by tensor-product quadrature."""
    x, wx = leggauss(n_rho)
    rho = 0.5 * R_g * (x + 1.0)
    wr = 0.5 * R_g * wx * rho ** (gamma + d - 1)
    pts, wp = _sphere(d, n_sph)
    area = wp.sum()
    gains, losses = [], []
    for vv in np.atleast_2d(v):
        gsum = 0.0
        lsum = 0.0
        for i in range(n_rho):
            base = vv[None, :] - 0.5 * rho[i] * pts  # v - g/2 for every ghat
            lsum += wr[i] * (wp * mixture_eval(params, vv[None, :] - rho[i] * pts)).sum()
            half = 0.5 * rho[i] * pts  # rho sigma / 2 for every sigma
            a = mixture_eval(params, base[:, None, :] + half[None, :, :])
            b = mixture_eval(params, base[:, None, :] - half[None, :, :])
            gsum += wr[i] * (wp[:, None] * wp[None, :] * a * b).sum()
        gains.append(gsum)
        losses.append(mixture_eval(params, vv[None, :])[0] * area * lsum)
    return np.array(gains), np.array(losses)
