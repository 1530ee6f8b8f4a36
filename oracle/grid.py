"""Velocity grid and quadrature rules (oracle; test infrastructure only).

Section 2.2: the velocity domain is truncated to [-L, L]^d, made periodic, and
sampled at k*dv with k in {-N/2+1, ..., N/2}; all quadrature weights equal the
volume dv^d of one grid cell.  Section 4.2: the spectral method assumes support
in B(0, R) with L = (3 sqrt 2 + 1) R / 2.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from numpy.polynomial.legendre import leggauss


@dataclass
class Spec:
    """Discretisation of one velocity cell.

    d        velocity dimension (2 or 3)
    N        points per axis
    L        half-width of the periodic box
    gamma    VHS exponent, B = |g|^gamma (gamma=0: Maxwell molecules, B = 1)
    n_theta  3D: Gauss-Legendre nodes in cos(theta) of the sigma rule
    n_phi    3D: uniform azimuth nodes;  2D: number of circle directions
    n_rho    Gauss-Legendre nodes of the radial |g| rule on [0, R_g]
    R        support radius; default from L = (3 sqrt 2 + 1) R / 2
    v1_shift physical v_1 of the grid's origin: the grid samples v' = v - v1_shift e_1.
             The collision operator and the discrete Maxwellian are translation
             invariant and work in v'; transport uses the physical v_1 = v'_1 + v1_shift.
    """

    d: int = 3
    N: int = 16
    L: float = 8.0
    gamma: float = 0.0
    n_theta: int = 4
    n_phi: int = 8
    n_rho: int = 8
    R: float | None = None
    v1_shift: float = 0.0
    _cache: dict = field(default_factory=dict, repr=False, compare=False)

    @property
    def dv(self) -> float:
        return 2.0 * self.L / self.N

    @property
    def w(self) -> float:
        """Equal quadrature weight dv^d (eq. velo_integral with uniform grid)."""
        return self.dv ** self.d

    @property
    def K(self) -> int:
        return self.N ** self.d

    @property
    def support_R(self) -> float:
        if self.R is not None:
            return self.R
        return 2.0 * self.L / (3.0 * np.sqrt(2.0) + 1.0)

    @property
    def R_g(self) -> float:
        """Truncation of the relative speed |v - v_*| <= 2R."""
        return 2.0 * self.support_R

    @property
    def M(self) -> int:
        return self.n_theta * self.n_phi if self.d == 3 else self.n_phi


def axis_nodes(spec: Spec) -> np.ndarray:
    """k * dv, k = -N/2+1 .. N/2 (Section 2.2)."""
    return (np.arange(spec.N) - spec.N // 2 + 1) * spec.dv


def velocity_nodes(spec: Spec) -> np.ndarray:
    """All K nodes as a [K, d] array in C order (axis 0 slowest)."""
    x = axis_nodes(spec)
    axes = np.meshgrid(*([x] * spec.d), indexing="ij")
    return np.stack([a.reshape(-1) for a in axes], axis=1)


def transport_v1(spec: Spec) -> np.ndarray:
    """Physical v_1 = v'_1 + v1_shift at every node (the advection speed along x)."""
    return velocity_nodes(spec)[:, 0] + spec.v1_shift


def phi_vectors(spec: Spec) -> np.ndarray:
    """Collision invariants phi(v) = (1, v_1..v_d, |v|^2) at every node, [K, d+2]."""
    v = velocity_nodes(spec)
    return np.concatenate([np.ones((v.shape[0], 1)), v, (v * v).sum(1, keepdims=True)], axis=1)


def sphere_rule(spec: Spec):
    """Directions sigma_p and weights w_p on S^{d-1} (sum w_p = |S^{d-1}|).

    3D: Gauss-Legendre in cos(theta) (n_theta) times uniform azimuth
    phi_j = 2 pi j / n_phi; sigma = (cos t, sin t cos phi, sin t sin phi), so the
    polar axis is velocity axis 0.  2D: theta_p = 2 pi p / n_phi, equal weights.
    Both rules are antipodally symmetric for even node counts."""
    if spec.d == 3:
        c, wc = leggauss(spec.n_theta)
        ph = 2.0 * np.pi * np.arange(spec.n_phi) / spec.n_phi
        sig, wts = [], []
        for ci, wi in zip(c, wc):
            st = np.sqrt(max(0.0, 1.0 - ci * ci))
            for p in ph:
                sig.append((ci, st * np.cos(p), st * np.sin(p)))
                wts.append(wi * 2.0 * np.pi / spec.n_phi)
        return np.array(sig), np.array(wts)
    th = 2.0 * np.pi * np.arange(spec.n_phi) / spec.n_phi
    return np.stack([np.cos(th), np.sin(th)], axis=1), np.full(spec.n_phi, 2.0 * np.pi / spec.n_phi)


def radial_rule(spec: Spec, n: int | None = None):
    """Gauss-Legendre nodes and weights on [0, R_g]."""
    n = spec.n_rho if n is None else n
    x, wx = leggauss(n)
    a = spec.R_g
    return 0.5 * a * (x + 1.0), 0.5 * a * wx


def sphere_area(d: int) -> float:
    """|S^{d-1}|: 2 (d=1, the two points +-1), 2 pi (d=2), 4 pi (d=3)."""
    return {1: 2.0, 2: 2.0 * np.pi, 3: 4.0 * np.pi}[d]


def S_d(d: int, z):
    """Integral of exp(i z e.sigma) over the unit sphere S^{d-1}:
    2 pi J_0(z) for d=2, 4 pi sin(z)/z for d=3."""
    z = np.asarray(z, dtype=np.float64)
    if d == 3:
        return 4.0 * np.pi * np.sinc(z / np.pi)
    from scipy.special import j0

    return 2.0 * np.pi * j0(z)


def frequencies(spec: Spec):
    """Signed DFT frequencies l (numpy FFT order) and xi_l = pi l / L per axis."""
    l = np.fft.fftfreq(spec.N) * spec.N
    return l, np.pi * l / spec.L


def xi_grids(spec: Spec):
    """Per-axis xi arrays broadcast to the full d-dimensional spectrum."""
    _, xi = frequencies(spec)
    return np.meshgrid(*([xi] * spec.d), indexing="ij")


def nyquist_mask(spec: Spec) -> np.ndarray:
    """True where any axis frequency equals -N/2 (the unpaired Nyquist mode)."""
    l, _ = frequencies(spec)
    ny = l == -spec.N // 2
    grids = np.meshgrid(*([ny] * spec.d), indexing="ij")
    m = np.zeros_like(grids[0])
    for g in grids:
        m = m | g
    return m
