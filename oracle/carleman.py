"""Carleman fast spectral form for hard spheres in 3D (oracle; test
infrastructure only).

The paper evaluates Q[f,f] with the Fourier spectral method of its cited
fast-spectral references (Section 2.2, Section 4.2).  For kernels that are
separable in the Carleman representation, that family has a fast form whose
cost has no radial quadrature factor.  In 3D the hard-sphere kernel
B = |g| (gamma = 1) is such a kernel.  Derivation used here:

  Carleman representation of the gain term (x = v' - v, y = v'_* - v, x.y = 0):
      Q+(v) = int int 4 |x + y|^{gamma - 1} delta(x.y) f(v + x) f(v + y) dx dy,
  so for gamma = 1 the weight is the constant 4.  x and y are each truncated to
  the ball of radius R_c = sqrt(2) R, R the support radius of f: in the cited
  fast spectral construction that truncation is free of aliasing exactly when
  L >= (3 sqrt 2 + 1) R / 2, the relation between L and R that Section 4.2
  fixes.  With x = rho e, the spectral weight of (l, m) is
      beta(l, m) = 4 int_{S^2_+} psi1(xi_l . e) Phi2(|P_e xi_m|) de,
      psi1(s) = 2 int_0^{R_c} rho cos(rho s) d rho            (e and -e folded)
      Phi2(t) = int_{y perp e, |y| <= R_c} exp(i xi.y) dy = 2 pi R_c J1(R_c t) / t,
  P_e the projection onto the plane perpendicular to e.  A quadrature of the
  half sphere (nodes e_p, weights w_p) gives the rank-M' form
      Q+(v) = sum_p a_p(v) b_p(v),   a_p = IDFT(A_p fh),  b_p = IDFT(B_p fh),
      A_p(xi) = 4 w_p psi1(xi . e_p),  B_p(xi) = Phi2(|P_{e_p} xi|),
  and the loss uses the same quadrature on the diagonal:
      Q-(v) = f(v) IDFT(beta(m, m) fh_m),  beta(m, m) = sum_p A_p(m) B_p(m).
  Since A_p and B_p are even, beta(l, -l) = beta(l, l), so the discrete form
  conserves mass exactly.  Nyquist coefficients of f are zeroed as in the
  sigma form (``collision.spectrum``).
"""
from __future__ import annotations

import numpy as np
from scipy.special import j1

from .collision import spectrum
from .grid import Spec, sphere_rule, xi_grids


def carleman_radius(spec: Spec) -> float:
    """Truncation radius R_c = sqrt(2) R of x and y (R the support radius)."""
    return np.sqrt(2.0) * spec.support_R


def half_sphere_rule(spec: Spec):
    """The directions of the sigma rule with cos(theta) > 0 (n_theta even) and
    their weights; the weights sum to 2 pi, the area of the half sphere."""
    if spec.d != 3 or spec.n_theta % 2:
        raise ValueError("the Carleman form needs d = 3 and an even n_theta")
    sig, w = sphere_rule(spec)
    keep = sig[:, 0] > 0.0
    return sig[keep], w[keep]


def psi1(spec: Spec, s):
    """2 int_0^{R_c} rho cos(rho s) d rho = 2 R_c^2 (x sin x + cos x - 1) / x^2,
    x = R_c s; a Taylor series below |x| = 0.5 avoids the cancellation."""
    Rc = carleman_radius(spec)
    x = np.asarray(Rc * np.asarray(s, dtype=np.float64))
    out = np.empty_like(x)
    small = np.abs(x) < 0.5
    xs = x[small]
    # sum_n (-1)^n x^{2n} (2n + 1) / (2n + 2)!
    ser = np.zeros_like(xs)
    term_fact = 2.0  # (2n + 2)! for n = 0
    for n in range(12):
        if n > 0:
            term_fact *= (2 * n + 1) * (2 * n + 2)
        ser += (-1) ** n * xs ** (2 * n) * (2 * n + 1) / term_fact
    out[small] = ser
    xb = x[~small]
    out[~small] = (xb * np.sin(xb) + np.cos(xb) - 1.0) / (xb * xb)
    return 2.0 * Rc * Rc * out


def phi2(spec: Spec, t):
    """2 pi R_c J1(R_c t) / t, equal to pi R_c^2 at t = 0."""
    Rc = carleman_radius(spec)
    x = np.asarray(Rc * np.asarray(t, dtype=np.float64))
    out = np.full_like(x, 0.5)
    nz = x > 1e-12
    out[nz] = j1(x[nz]) / x[nz]
    return 2.0 * np.pi * Rc * Rc * out


def direction_weights(spec: Spec):
    """A_p and B_p on the spectrum grid for every half-sphere direction:
    two arrays [M', N, N, N]."""
    e, w = half_sphere_rule(spec)
    xg = xi_grids(spec)
    x2 = sum(a * a for a in xg)
    A, B = [], []
    for ep, wp in zip(e, w):
        s = xg[0] * ep[0] + xg[1] * ep[1] + xg[2] * ep[2]
        t = np.sqrt(np.maximum(x2 - s * s, 0.0))
        A.append(4.0 * wp * psi1(spec, s))
        B.append(phi2(spec, t))
    return np.array(A), np.array(B)


def q_carleman(spec: Spec, f: np.ndarray, parts: bool = False):
    """Q[f, f] by the rank-M' Carleman form, direction by direction."""
    if spec.gamma != 1.0:
        raise ValueError("the Carleman form is for hard spheres (gamma = 1)")
    K = spec.K
    fh = spectrum(spec, f)
    A, B = direction_weights(spec)
    gain = np.zeros(K)
    for Ap, Bp in zip(A, B):
        a = (np.fft.ifftn(Ap * fh) * K).real.reshape(-1)
        b = (np.fft.ifftn(Bp * fh) * K).real.reshape(-1)
        gain += a * b
    beta = (A * B).sum(0)
    loss = f * (np.fft.ifftn(beta * fh) * K).real.reshape(-1)
    if parts:
        return gain, loss
    return gain - loss


# ---------------------------------------------------------------- 2D, Maxwell molecules
# In two dimensions the Carleman weight of B = |g|^gamma is 2 |x + y|^gamma, the
# constant 2 for Maxwell molecules (gamma = 0).  With x = rho e over the half
# circle (rho of either sign) and y perpendicular to x, y = rho' e_perp, the
# delta(x.y) integral cancels the Jacobian |rho| of x, so
#     Q+(v) = 2 int_{half circle} de int int f(v + rho e) f(v + rho' e_perp) drho drho'.
# Truncating rho and rho' to [-R_c, R_c] (R_c = sqrt(2) R, as in 3D), the shift
# integrals are psi2(xi.e) and psi2(xi.e_perp) with
#     psi2(s) = int_{-R_c}^{R_c} exp(i rho s) drho = 2 R_c sinc(R_c s),
# so a half-circle rule (nodes e_p, weights w_p) gives the rank-M/2 form
#     Q+ = sum_p IDFT(A_p fh) IDFT(B_p fh),  A_p = 2 w_p psi2(xi.e_p),  B_p = psi2(xi.e_p_perp),
# and the loss f IDFT(beta fh) with beta = sum_p A_p B_p, which conserves mass
# exactly (A_p, B_p even).  The half-circle rule is the circle rule's nodes
# theta_p = 2 pi p / M with p < M / 2 and weights 2 pi / M (they sum to pi).


def psi2(spec: Spec, s):
    """int_{-R_c}^{R_c} exp(i rho s) drho = 2 R_c sinc(R_c s)."""
    Rc = carleman_radius(spec)
    return 2.0 * Rc * np.sinc(Rc * np.asarray(s, dtype=np.float64) / np.pi)


def direction_weights_2d(spec: Spec):
    """A_p and B_p on the 2D spectrum grid: two arrays [M/2, N, N]."""
    M = spec.n_phi
    xg = xi_grids(spec)
    A, B = [], []
    for p in range(M // 2):
        t = 2.0 * np.pi * p / M
        e, ep = (np.cos(t), np.sin(t)), (-np.sin(t), np.cos(t))
        wp = 2.0 * np.pi / M
        A.append(2.0 * wp * psi2(spec, xg[0] * e[0] + xg[1] * e[1]))
        B.append(psi2(spec, xg[0] * ep[0] + xg[1] * ep[1]))
    return np.array(A), np.array(B)


def q_carleman_2d(spec: Spec, f: np.ndarray, parts: bool = False):
    """Q[f, f] for 2D Maxwell molecules by the rank-M/2 Carleman form."""
    if spec.d != 2 or spec.gamma != 0.0 or spec.n_phi % 2:
        raise ValueError("the 2D Carleman form is for Maxwell molecules (gamma = 0) on an even circle rule")
    K = spec.K
    fh = spectrum(spec, f)
    A, B = direction_weights_2d(spec)
    gain = np.zeros(K)
    for Ap, Bp in zip(A, B):
        a = (np.fft.ifftn(Ap * fh) * K).real.reshape(-1)
        b = (np.fft.ifftn(Bp * fh) * K).real.reshape(-1)
        gain += a * b
    beta = (A * B).sum(0)
    loss = f * (np.fft.ifftn(beta * fh) * K).real.reshape(-1)
    if parts:
        return gain, loss
    return gain - loss
