"""Fourier-spectral collision operator (oracle; test infrastructure only).

Section 2.2 evaluates Q[f,f] of eq. collision with the Fourier spectral
method on the periodic box [-L, L)^d, and uses the steady-state preserving
form of eq. discrete_Q.  Section 4.2 fixes Maxwell molecules B = 1 and the
support radius R with L = (3 sqrt 2 + 1) R / 2.

Derivation used here (sigma-representation of eq. collision, periodic f,
relative speed truncated at R_g = 2R, B = |g|^gamma):
  f(v) = sum_l fh_l exp(i xi_l.v),   xi_l = pi l / L,
  gain  Qh+_k = sum_{l+m=k} fh_l fh_m G(l, m),
        G(l,m) = int_0^{R_g} rho^{gamma+d-1} S_d(rho|xi_l+xi_m|/2)
                 int_{S^{d-1}} exp(i rho (xi_l - xi_m).sigma / 2) dsigma drho,
  loss  Q-(v) = f(v) sum_m Gm(m) fh_m exp(i xi_m.v),
        Gm(m) = |S^{d-1}| int_0^{R_g} rho^{gamma+d-1} S_d(rho |xi_m|) drho,
with S_d(z) the integral of exp(i z e.sigma) over the sphere.

Two evaluations:
  * ``q_fsm``: the fast form.  The sigma integral uses an M-point rule and the
    radial one an n_rho-point Gauss rule.  Then the l,m dependence separates
    into shifted copies a = f(v + s), b = f(v - s), s = rho sigma / 2, and
    the convolution is the DFT of the pointwise product a*b.  It loops over
    every one of the M directions, with no pairing or reuse.
  * ``q_direct``: the sigma-exact spectral sum D (the sigma integral done in
    closed form, S_d(rho |xi_l - xi_m| / 2)), by an O(K^2) sum over (k, l).
    It is for tiny grids, and the fast form converges to it as M, n_rho grow.
The Nyquist coefficients (any axis index -N/2) of f are zeroed in both, so
shifted copies of a real f stay real.
"""
from __future__ import annotations

import numpy as np

from .grid import Spec, S_d, frequencies, nyquist_mask, phi_vectors, radial_rule, sphere_area, sphere_rule, xi_grids
from .maxwellian import discrete_maxwellian, moments


def spectrum(spec: Spec, f: np.ndarray) -> np.ndarray:
    """DFT coefficients fh with f(v_j) = sum_l fh_l e^{i xi_l.(v_j - v_0)}; Nyquist zeroed."""
    F = np.fft.fftn(f.reshape((spec.N,) * spec.d)) / spec.K
    F[nyquist_mask(spec)] = 0.0
    return F


def _xi_norm(spec: Spec) -> np.ndarray:
    g = xi_grids(spec)
    return np.sqrt(sum(x * x for x in g))


def gain_weights(spec: Spec):
    """W_r(|xi_k|) = w_r rho_r^{gamma+d-1} S_d(rho_r |xi_k| / 2), one array per radial node."""
    rho, wr = radial_rule(spec)
    xn = _xi_norm(spec)
    return [wr[i] * rho[i] ** (spec.gamma + spec.d - 1) * S_d(spec.d, rho[i] * xn / 2.0) for i in range(len(rho))]


def loss_weight(spec: Spec, n_rho: int | None = None) -> np.ndarray:
    """Gm(|xi_m|) = |S^{d-1}| int_0^{R_g} rho^{gamma+d-1} S_d(rho|xi_m|) drho with the
    same radial rule as the gain (or an n_rho-point rule when given)."""
    rho, wr = radial_rule(spec, n_rho)
    xn = _xi_norm(spec)
    out = np.zeros_like(xn)
    for i in range(len(rho)):
        out += wr[i] * rho[i] ** (spec.gamma + spec.d - 1) * S_d(spec.d, rho[i] * xn)
    return sphere_area(spec.d) * out


def q_fsm(spec: Spec, f: np.ndarray, parts: bool = False):
    """Q^FSM[f, f] by the fast sigma-form (all M directions, one by one)."""
    N, d = spec.N, spec.d
    fh = spectrum(spec, f)
    xis = xi_grids(spec)
    sig, wsig = sphere_rule(spec)
    rho, _ = radial_rule(spec)
    W = gain_weights(spec)
    Qh = np.zeros((N,) * d, dtype=np.complex128)
    for i in range(len(rho)):
        acc = np.zeros((N,) * d)
        for p in range(len(wsig)):
            s = rho[i] * sig[p] / 2.0
            ph = np.exp(1j * sum(xis[a] * s[a] for a in range(d)))
            a_ = np.fft.ifftn(fh * ph).real * spec.K
            b_ = np.fft.ifftn(fh * np.conj(ph)).real * spec.K
            acc += wsig[p] * a_ * b_
        Qh += W[i] * np.fft.fftn(acc) / spec.K
    gain = (np.fft.ifftn(Qh) * spec.K).real.reshape(-1)
    Lf = (np.fft.ifftn(loss_weight(spec) * fh) * spec.K).real.reshape(-1)
    loss = f * Lf
    if parts:
        return gain, loss
    return gain - loss


def q_direct(spec: Spec, f: np.ndarray, n_rho_exact: int = 64, parts: bool = False):
    """sigma-exact spectral sum D: Qh+_k = sum_l fh_l fh_m W(k,l,m), m = k - l (mod N),
    W = int rho^{gamma+d-1} S_d(rho |xi_k|/2) S_d(rho |xi_l - xi_m| / 2) drho with a
    high-order radial rule.  O(K^2 n_rho); tiny grids only."""
    N, d, K = spec.N, spec.d, spec.K
    fh = spectrum(spec, f).reshape(-1)
    l1, xi1 = frequencies(spec)
    idx = np.array(np.unravel_index(np.arange(K), (N,) * d)).T  # [K, d] axis indices
    xi = xi1[idx]  # [K, d]
    xk = np.linalg.norm(xi, axis=1)
    rho, wr = radial_rule(spec, n_rho_exact)
    wrad = wr * rho ** (spec.gamma + d - 1)
    Qh = np.zeros(K, dtype=np.complex128)
    for k in range(K):
        m_idx = (idx[k][None, :] - idx) % N  # [K, d]
        m_flat = np.ravel_multi_index(m_idx.T, (N,) * d)
        diff = np.linalg.norm(xi - xi1[m_idx], axis=1)  # |xi_l - xi_m| with signed freqs
        # W(k, l, m) for every l at once
        Wk = (S_d(d, np.outer(diff, rho) / 2.0) * (S_d(d, rho * xk[k] / 2.0) * wrad)[None, :]).sum(1)
        Qh[k] = np.sum(fh * fh[m_flat] * Wk)
    gain = (np.fft.ifftn(Qh.reshape((N,) * d)) * K).real.reshape(-1)
    Lf = (np.fft.ifftn(loss_weight(spec, n_rho_exact) * fh.reshape((N,) * d)) * K).real.reshape(-1)
    loss = f * Lf
    if parts:
        return gain, loss
    return gain - loss


def mass_project(spec: Spec, Q: np.ndarray, M: np.ndarray) -> np.ndarray:
    """Q - M (sum_k Q_k) / (sum_k M_k): removes, along the Maxwellian, the mass the
    sigma quadrature of the gain term creates.  With diffuse walls the only
    globally conserved quantity is mass: summing the discrete residual over all
    cells gives -(1/eps) sum_j dx sum_k w Q_jk, so a steady state exists only if
    that vanishes."""
    return Q - M * (np.sum(Q) / np.sum(M))


def conserve_project(spec: Spec, Q: np.ndarray, M: np.ndarray) -> np.ndarray:
    """Q - M (phi . a) with sum_k phi_i M phi_j a_j = sum_k phi_i Q_k, phi = (1, v, |v|^2):
    removes, along M times the collision invariants, the mass, momentum and
    energy that the discrete operator creates (sigma quadrature, truncation and
    periodisation of the spectral method), so that it conserves all five to
    rounding, as the collision integral does.  It is the change of least
    sum_k dQ_k^2 / M_k.  Summing the discrete residual over all cells leaves
    -(1/eps) sum_j dx sum_k w phi Q_jk plus the boundary fluxes; with inflow at
    both ends every invariant is balanced, so a steady state exists only if this
    sum vanishes."""
    phi = phi_vectors(spec)
    G = (phi * M[:, None]).T @ phi
    a = np.linalg.solve(G, phi.T @ Q)
    return Q - M * (phi @ a)


def q_corrected(spec: Spec, f: np.ndarray, M: np.ndarray | None = None, op=q_fsm, conserve: str | None = None):
    """Steady-state preserving collision term, eq. discrete_Q:
    Q[f] = Q^FSM[f, f] - Q^FSM[M[f], M[f]]; then, with conserve = "mass" or "all",
    mass_project or conserve_project."""
    if M is None:
        M = discrete_maxwellian(spec, f)
    Q = op(spec, f) - op(spec, M)
    if conserve == "mass":
        return mass_project(spec, Q, M)
    if conserve == "all":
        return conserve_project(spec, Q, M)
    return Q


def pair_speed_moment(spec: Spec, T: float) -> float:
    """<|g|^gamma> over pairs drawn from a Maxwellian of temperature T.  The
    relative velocity of two such particles is Maxwellian with temperature 2T,
    so |g|^2 / (2T) is chi-squared with d degrees of freedom and
    <|g|^gamma> = (4T)^{gamma/2} Gamma((d + gamma)/2) / Gamma(d/2); it is 1 for
    gamma = 0."""
    from math import gamma as Gamma

    g, d = spec.gamma, spec.d
    return (4.0 * T) ** (g / 2.0) * Gamma((d + g) / 2.0) / Gamma(d / 2.0)


def nu_of(spec: Spec, f: np.ndarray, theta: np.ndarray | None = None) -> float:
    """BGK-penalty frequency of eq. Pf: nu = |S^{d-1}| rho <|g|^gamma>, the binary
    loss frequency averaged over pairs from the cell's Maxwellian, with T the
    temperature parameter 1 / (2 theta_gamma) of the discrete Maxwellian.  For
    Maxwell molecules (gamma = 0) this is |S^{d-1}| rho: 2 pi rho for 2D velocity
    (Section 4.2), 4 pi rho in 3D (Section 4.1.2), where the BGK loss matches
    the binary loss exactly; for hard spheres the average keeps the penalty of
    the same size as the loss term it stands in for."""
    rho = moments(spec, f)[0]
    if spec.gamma == 0.0:
        return sphere_area(spec.d) * rho
    if theta is None:
        theta = discrete_maxwellian(spec, f, return_theta=True)[1]
    return sphere_area(spec.d) * rho * pair_speed_moment(spec, 0.5 / theta[-1])


def bgk_nu_of(spec: Spec, f: np.ndarray) -> float:
    """Collision frequency of the BGK model: |S^{d-1}| rho (Section 4.1.2)."""
    return sphere_area(spec.d) * moments(spec, f)[0]


def penalty_split(Q: np.ndarray, M: np.ndarray, f: np.ndarray, nu) -> np.ndarray:
    """P = Q - nu (M - f), eq. Pf: the part of the collision term that the scans
    treat explicitly (Section 3.3).  Broadcasts nu over the trailing velocity axis."""
    return Q - np.asarray(nu)[..., None] * (M - f)


def penalty(spec: Spec, f: np.ndarray, Q: np.ndarray | None = None, M: np.ndarray | None = None,
            conserve: str | None = "mass"):
    """P[f] = Q[f,f] - nu (M[f] - f), eq. Pf, with the mass-projected corrected Q."""
    if M is None:
        M = discrete_maxwellian(spec, f)
    if Q is None:
        Q = q_corrected(spec, f, M, conserve=conserve)
    return penalty_split(Q, M, f, nu_of(spec, f))
