"""Pins of the oracle's two-dimensional velocity operator (d = 2; CPU only).

The paper's binary-collision runs use two-dimensional velocities and Maxwell
molecules (Section 4.2).  Each test checks the oracle against something other
than itself: the 2D BKW closed form, an independent physical-space quadrature,
exact mass conservation of the sigma-exact sum, convergence of the fast form to
that sum, and exactness of the corrected form at equilibrium."""
import numpy as np

import synth
from oracle import collision as C, maxwellian as MX, physical as PH
from oracle.grid import Spec, velocity_nodes


def _sp(N, L=8.0, M=16, nr=8, gamma=0.0):
    return Spec(d=2, N=N, L=L, n_phi=M, n_rho=nr, gamma=gamma)


def test_bkw_closed_form_2d():
    # 2D Bobylev-Krook-Wu solution for Maxwell molecules with the kernel
    # normalised to one over the circle: f = exp(-v^2/2K)/(2 pi K^2) (2K - 1 +
    # (1 - K) v^2 / (2K)), K = 1 - exp(-t/8)/2, and Q[f] = df/dt.  With B = 1 the
    # operator is 2 pi times that.  The error must fall as the grid is refined.
    t = 1.0
    K = 1.0 - 0.5 * np.exp(-t / 8.0)
    dK = np.exp(-t / 8.0) / 16.0
    errs = []
    for N, M, nr in [(24, 16, 12), (48, 32, 24)]:
        sp = _sp(N, M=M, nr=nr)
        v2 = (velocity_nodes(sp) ** 2).sum(1)
        E = np.exp(-v2 / (2 * K))
        poly = 2 * K - 1 + (1 - K) * v2 / (2 * K)
        f = E / (2 * np.pi * K * K) * poly
        # d/dK of f, times dK/dt
        dpoly = 2 - v2 / (2 * K * K)
        df = (E / (2 * np.pi * K * K) * (v2 / (2 * K * K) * poly - 2 / K * poly + dpoly)) * dK
        Q = C.q_fsm(sp, f)
        ref = 2 * np.pi * df
        errs.append(np.abs(Q - ref).max() / np.abs(ref).max())
    assert errs[1] < 0.1 * errs[0]
    assert errs[1] < 1e-4


def test_fast_form_matches_physical_space_quadrature_2d():
    N, L = 32, 8.0
    sp = _sp(N, L, M=32, nr=16)
    rng = np.random.default_rng([6, 0])
    params = synth.mixture_params(rng, d=2, T=(0.8, 1.2), speed=(0.0, 0.5))
    f = synth.maxwellian_mixture(params, N, L, d=2)
    g, l = C.q_fsm(sp, f, parts=True)
    v = velocity_nodes(sp)
    idx = [i for i in range(len(v)) if np.linalg.norm(v[i]) < 1.9][::7][:4]
    gp, lp = PH.q_physical(params, v[idx], 2, sp.R_g, n_rho=48, n_sph=48)
    scale = np.abs(l).max()
    assert np.max(np.abs(g[idx] - gp)) < 1e-7 * scale
    assert np.max(np.abs(l[idx] - lp)) < 1e-7 * scale


def test_sigma_exact_sum_conserves_mass_2d():
    sp = _sp(12, 4.0)
    f = synth.mixture_batch(1, 12, 4.0, d=2, seed=3, T=(0.15, 0.25), speed=(0.0, 0.3))[0]
    D = C.q_direct(sp, f)
    _, l = C.q_direct(sp, f, parts=True)
    assert abs(MX.moments(sp, D)[0]) < 1e-13 * sp.w * np.abs(l).sum()


def test_fast_form_converges_to_sigma_exact_sum_2d():
    f = synth.mixture_batch(1, 12, 4.0, d=2, seed=3, T=(0.15, 0.25), speed=(0.0, 0.3))[0]
    D = C.q_direct(_sp(12, 4.0), f)
    errs = []
    for M, nr in ((8, 4), (16, 8), (32, 16)):
        errs.append(np.abs(C.q_fsm(_sp(12, 4.0, M=M, nr=nr), f) - D).max() / np.abs(D).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-10


def test_maxwellian_equilibrium_and_corrected_form_2d():
    sp = _sp(32, M=16, nr=8)
    f = synth.mixture_batch(1, 32, 8.0, d=2, seed=2, T=(0.8, 1.2), speed=(0.0, 0.3))[0]
    M = MX.discrete_maxwellian(sp, f)
    m_f, m_M = MX.moments(sp, f), MX.moments(sp, M)
    assert np.abs(m_f - m_M).max() < 1e-13 * np.abs(m_f).max()
    g, l = C.q_fsm(sp, M, parts=True)
    assert np.abs(g - l).max() < 1e-6 * np.abs(l).max()
    assert np.abs(C.q_corrected(sp, M, M)).max() == 0.0
