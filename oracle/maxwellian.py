"""Moments and the discrete Maxwellian (oracle; test infrastructure only).

eq. moment: rho, U, T of f.  eqs. discrete_conservation / discrete_Gaussian:
the discrete Maxwellian exp(alpha + beta.v - gamma |v|^2) whose discrete
moments against phi = (1, v, |v|^2) equal those of f, found by Newton's
method (Section 2.2).  All sums are plain O(K) sums over the grid.
"""
from __future__ import annotations

import numpy as np

from .grid import Spec, phi_vectors, velocity_nodes


def moments(spec: Spec, f: np.ndarray) -> np.ndarray:
    """Discrete moments sum_k w phi(v_k) f_k, shape [d+2]."""
    return spec.w * phi_vectors(spec).T @ f


def macroscopic(spec: Spec, f: np.ndarray):
    """rho, U, T from the discrete moments (eq. moment)."""
    m = moments(spec, f)
    rho = m[0]
    U = m[1 : 1 + spec.d] / rho
    T = (m[-1] / rho - U @ U) / spec.d
    return rho, U, T


def theta_from_macro(spec: Spec, rho, U, T) -> np.ndarray:
    """Parameters of the continuous Maxwellian written as exp(alpha + beta.v - gamma|v|^2)
    (eq. maxwellian rewritten in the form of eq. discrete_Gaussian)."""
    d = spec.d
    U = np.asarray(U, dtype=np.float64)
    alpha = np.log(rho / (2.0 * np.pi * T) ** (d / 2.0)) - (U @ U) / (2.0 * T)
    return np.concatenate([[alpha], U / T, [1.0 / (2.0 * T)]])


def gaussian(spec: Spec, theta: np.ndarray) -> np.ndarray:
    """exp(alpha + beta.v - gamma |v|^2) at every node (eq. discrete_Gaussian)."""
    v = velocity_nodes(spec)
    d = spec.d
    return np.exp(theta[0] + v @ theta[1 : 1 + d] - theta[-1] * (v * v).sum(1))


def _phi_tilde(spec: Spec) -> np.ndarray:
    """d/dtheta of (alpha + beta.v - gamma|v|^2): (1, v, -|v|^2)."""
    p = phi_vectors(spec).copy()
    p[:, -1] *= -1.0
    return p


def solve_weighted_gaussian(spec: Spec, target: np.ndarray, weight: np.ndarray | None = None,
                            theta0: np.ndarray | None = None, tol: float = 1e-13, max_iter: int = 60):
    """Newton's method for sum_k w c_k phi_k exp(theta.phi~_k) = target.

    c_k = weight (1 when None).  With c = 1 this is the discrete Maxwellian
    (eq. discrete_conservation); with c = |v_1|/dx it is step 1 of the
    preconditioned iteration (eq. step1).  Backtracking halves the step while
    the residual grows.  Returns (theta, iterations, converged)."""
    phi = phi_vectors(spec)
    pt = _phi_tilde(spec)
    c = np.ones(spec.K) if weight is None else weight
    v = velocity_nodes(spec)
    if theta0 is None:
        # initial guess from the continuous moments of the target, read as a plain density
        rho = target[0]
        U = target[1 : 1 + spec.d] / rho
        T = max((target[-1] / rho - U @ U) / spec.d, 1e-3)
        theta = theta_from_macro(spec, rho, U, T)
    else:
        theta = np.array(theta0, dtype=np.float64)
    scale = np.abs(target[0]) + np.abs(target[-1]) + 1e-300

    def F(th):
        # a trial step may overflow; the backtracking below rejects non-finite residuals
        with np.errstate(over="ignore", invalid="ignore"):
            g = np.exp(th[0] + v @ th[1 : 1 + spec.d] - th[-1] * (v * v).sum(1))
            return spec.w * phi.T @ (c * g) - target, g

    r, g = F(theta)
    nrm = np.max(np.abs(r))
    for it in range(max_iter):
        if nrm <= tol * scale:
            return theta, it, True
        J = spec.w * (phi * (c * g)[:, None]).T @ pt
        if not np.isfinite(J).all():
            return theta, it, False
        try:
            step = np.linalg.solve(J, -r)
        except np.linalg.LinAlgError:
            # a singular Jacobian is a Newton failure, not an error of the caller
            return theta, it, False
        t = 1.0
        while True:
            th_new = theta + t * step
            r_new, g_new = F(th_new)
            n_new = np.max(np.abs(r_new))
            if np.isfinite(n_new) and (n_new < nrm or t < 1e-4) and th_new[-1] > 0.0:
                break
            t *= 0.5
            if t < 1e-6:
                break
        if np.max(np.abs(th_new - theta)) <= 1e-15 * (1.0 + np.max(np.abs(theta))):
            theta, r, g, nrm = th_new, r_new, g_new, n_new
            return theta, it + 1, nrm <= 1e-10 * scale
        theta, r, g, nrm = th_new, r_new, g_new, n_new
    return theta, max_iter, nrm <= tol * scale


def discrete_maxwellian(spec: Spec, f: np.ndarray, return_theta: bool = False):
    """M[f]: the discrete Gaussian with the same discrete moments as f
    (eqs. discrete_conservation, discrete_Gaussian; Newton, Section 2.2)."""
    theta, _, ok = solve_weighted_gaussian(spec, moments(spec, f))
    if not ok:
        raise RuntimeError("discrete Maxwellian Newton did not converge")
    M = gaussian(spec, theta)
    return (M, theta) if return_theta else M
