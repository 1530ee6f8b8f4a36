"""GPU parity of the two-dimensional velocity operator (d = 2) against the FP64
CPU oracle, through the C ABI: the sigma form, its steady-state corrected and
mass-projected forms, and the discrete Maxwellian."""
import numpy as np
import pytest

import synth
from oracle import collision as OQ, maxwellian as OM
from oracle.grid import Spec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_01910_amd as bz

    bz.load_library()
    return bz


def _T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


# (N, L, M, n_rho, gamma, batch): every transform length (radix 4, 3 and 2
# passes), ragged batches, Maxwell molecules and hard spheres
CASES = [(8, 4.0, 8, 4, 0.0, 3), (12, 6.0, 16, 6, 0.0, 5), (24, 8.0, 32, 12, 1.0, 2), (48, 8.0, 64, 24, 0.0, 2)]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("form", ["plain", "corrected", "mass"])
def test_eval_q_2d_matches_oracle(bz, case, form):
    N, L, M, nr, gam, B = case
    print(f"d=2 eval_Q N={N} M={M} n_rho={nr} gamma={gam} form={form}", flush=True)
    sp = Spec(d=2, N=N, L=L, n_phi=M, n_rho=nr, gamma=gam)
    f = synth.mixture_batch(B, N, L, d=2, seed=41)
    ctx = bz.Context(N=N, L=L, n_phi=M, n_rho=nr, gamma=gam, d=2)
    Q = ctx.eval_Q(_T(f), corrected=form != "plain", conserve="mass" if form == "mass" else None).cpu().numpy()
    for i in range(B):
        gain, loss = OQ.q_fsm(sp, f[i], parts=True)
        if form == "plain":
            ref = gain - loss
        else:
            ref = OQ.q_corrected(sp, f[i], conserve="mass" if form == "mass" else None)
        scale = max(np.abs(ref).max(), np.abs(loss).max())
        err = float(np.abs(Q[i] - ref).max() / scale)
        print(f"cell {i} rel err {err:.3e}", flush=True)
        assert err < 1e-12
        if form == "mass":
            assert abs(Q[i].sum()) < 1e-13 * np.abs(Q[i]).sum()


@pytest.mark.parametrize("N,L", [(8, 4.0), (24, 8.0), (48, 8.0)])
def test_maxwellian_2d_matches_oracle(bz, N, L):
    sp = Spec(d=2, N=N, L=L)
    f = synth.mixture_batch(4, N, L, d=2, seed=42)
    ctx = bz.Context(N=N, L=L, n_phi=8, n_rho=4, d=2)
    theta, M, it = ctx.maxwellian(_T(f))
    theta, M, it = theta.cpu().numpy(), M.cpu().numpy(), it.cpu().numpy()
    assert theta.shape == (4, 4)
    for i in range(4):
        Mo, tho = OM.discrete_maxwellian(sp, f[i], return_theta=True)
        assert it[i] >= 0
        assert np.abs(theta[i] - tho).max() < 1e-12 * (1 + np.abs(tho).max())
        assert np.abs(M[i] - Mo).max() < 1e-12 * Mo.max()


def test_full_size_2d_workload_matches_sampled_cells(bz):
    # the cavity's velocity discretisation: 4096 cells on 48^2 over [-8, 8]^2,
    # M = 64, n_rho = 24, corrected and mass-projected
    N, L, B = 48, 8.0, 4096
    print("d=2 full workload", flush=True)
    f = synth.mixture_batch(B, N, L, d=2, seed=0)
    ctx = bz.Context(N=N, L=L, n_phi=64, n_rho=24, d=2)
    Q = ctx.eval_Q(_T(f), corrected=True, conserve="mass")
    assert torch.isfinite(Q).all().item()
    mass = Q.sum(1).abs() / Q.abs().sum(1)
    assert mass.max().item() < 1e-12
    Qc = Q.cpu().numpy()
    sp = Spec(d=2, N=N, L=L, n_phi=64, n_rho=24)
    for i in (0, 4095):
        ref = OQ.q_corrected(sp, f[i], conserve="mass")
        _, loss = OQ.q_fsm(sp, f[i], parts=True)
        err = float(np.abs(Qc[i] - ref).max() / max(np.abs(ref).max(), np.abs(loss).max()))
        print(f"cell {i} rel err {err:.3e}", flush=True)
        assert err < 1e-12


def test_2d_context_refuses_what_it_does_not_implement(bz):
    ctx = bz.Context(N=8, L=4.0, n_phi=8, n_rho=4, d=2)
    f = _T(synth.mixture_batch(2, 8, 4.0, d=2, seed=1))
    with pytest.raises(bz.BZError):
        ctx.eval_Q(f, corrected=True, conserve="all")
    with pytest.raises(bz.BZError):
        ctx.cell_fixed_point(f, torch.zeros_like(f), _T(np.ones(2)), 0.1)
    with pytest.raises(bz.BZError):
        bz.Context(N=20, L=4.0, n_phi=8, n_rho=4, d=2)
    with pytest.raises(bz.BZError):
        bz.Context(N=8, L=4.0, n_phi=8, n_rho=4, d=2, method=bz.BZ_METHOD_CARLEMAN, gamma=1.0)


@pytest.mark.parametrize("N,L,M,nr", [(12, 6.0, 16, 6), (48, 8.0, 64, 24)])
def test_eval_q_2d_fp32_spectral_stage_within_stated_bound(bz, N, L, M, nr):
    # transforms, direction products and their accumulation in FP32; fields,
    # Maxwellian, loss combination and mass projection in FP64.  Bound: 2e-6 of
    # max(|Q|, |Q-|), as for the 3D FP32 stage
    B = 3
    sp = Spec(d=2, N=N, L=L, n_phi=M, n_rho=nr)
    f = synth.mixture_batch(B, N, L, d=2, seed=43)
    ctx = bz.Context(N=N, L=L, n_phi=M, n_rho=nr, d=2, precision=bz.BZ_FP32)
    Q = ctx.eval_Q(_T(f), corrected=True, conserve="mass").cpu().numpy()
    for i in range(B):
        ref = OQ.q_corrected(sp, f[i], conserve="mass")
        _, loss = OQ.q_fsm(sp, f[i], parts=True)
        err = float(np.abs(Q[i] - ref).max() / max(np.abs(ref).max(), np.abs(loss).max()))
        print(f"FP32 d=2 N={N} cell {i} rel err {err:.3e}", flush=True)
        assert err < 2e-6
        assert abs(Q[i].sum()) < 1e-13 * np.abs(Q[i]).sum()


@pytest.mark.parametrize("N,L,M,B", [(12, 6.0, 8, 3), (24, 8.0, 16, 2), (48, 8.0, 64, 2)])
@pytest.mark.parametrize("form", ["plain", "corrected", "mass"])
@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 2e-6)])
def test_carleman_2d_maxwell_matches_oracle(bz, N, L, M, B, form, prec, tol):
    from oracle import carleman as CA

    print(f"2D Carleman N={N} M={M} form={form} precision={prec}", flush=True)
    sp = Spec(d=2, N=N, L=L, n_phi=M)
    f = synth.mixture_batch(B, N, L, d=2, seed=44)
    ctx = bz.Context(N=N, L=L, n_phi=M, n_rho=2, d=2, method=bz.BZ_METHOD_CARLEMAN, precision=prec)
    Q = ctx.eval_Q(_T(f), corrected=form != "plain", conserve="mass" if form == "mass" else None).cpu().numpy()
    for i in range(B):
        gain, loss = CA.q_carleman_2d(sp, f[i], parts=True)
        if form == "plain":
            ref = gain - loss
        else:
            ref = OQ.q_corrected(sp, f[i], op=CA.q_carleman_2d, conserve="mass" if form == "mass" else None)
        err = float(np.abs(Q[i] - ref).max() / max(np.abs(ref).max(), np.abs(loss).max()))
        print(f"cell {i} rel err {err:.3e}", flush=True)
        assert err < tol
        if form == "plain" and prec == 0:  # exact mass conservation of the plain form
            assert abs(Q[i].sum()) < 1e-12 * np.abs(gain).sum()
