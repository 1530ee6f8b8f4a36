"""The remaining calls of the C ABI against the oracle or the plain calls:
bz_eval_Q_strided (row-strided views), bz_cell_fixed_point_ex (per-cell
penalty frequency, cell width and initial guess) and strict mode
(bz_set_strict, bz_cell_check)."""
import numpy as np
import pytest

import synth
from oracle import cell as OC, collision as OQ
from oracle.grid import Spec, velocity_nodes
from oracle.maxwellian import discrete_maxwellian

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


@pytest.mark.parametrize("N,d", [(8, 3), (16, 3), (24, 2)])
def test_strided_eval_q_equals_the_contiguous_call(bz, N, d):
    B = 5
    ctx = bz.Context(N=N, L=8.0, n_theta=2, n_phi=4, n_rho=3, d=d)
    K = ctx.K
    f = _T(synth.mixture_batch(B, N, 8.0, d=d, seed=7))
    Q = ctx.eval_Q(f, corrected=True, conserve="mass")
    big = torch.full((2 * B, K + 3), 7.0, dtype=torch.float64, device="cuda:0")
    big[::2, :K] = f
    fv = big[::2, :K]                  # rows 2 (K + 3) apart
    out_base = torch.full((3 * B, K), -1.0, dtype=torch.float64, device="cuda:0")
    out = out_base[::3]                # rows 3 K apart
    ctx.eval_Q_strided(fv, out, corrected=True, conserve="mass")
    assert torch.equal(out, Q)
    assert (out_base[1::3] == -1.0).all() and (out_base[2::3] == -1.0).all()  # rows between untouched
    assert (big[1::2] == 7.0).all() and (big[::2, K:] == 7.0).all()
    # unit strides: the plain call
    out2 = torch.empty_like(f)
    ctx.eval_Q_strided(f, out2, corrected=True, conserve="mass")
    assert torch.equal(out2, Q)
    with pytest.raises(bz.BZError):
        ctx.eval_Q_strided(big[::2, :K - 1], out)


def test_cell_fixed_point_ex_matches_oracle(bz):
    # given nu (not the matched frequency), per-cell widths and initial guesses
    N, L, nt, nph, nr, B = 8, 6.0, 2, 4, 3, 5
    sp = Spec(d=3, N=N, L=L, n_theta=nt, n_phi=nph, n_rho=nr)
    fo, fl, fr, eps = synth.cell_inflow_batch(B, N, L, 1 / 16, seed=41)
    rng = np.random.default_rng([41, 1])
    dxs = rng.uniform(1 / 32, 1 / 8, size=B)
    v1 = velocity_nodes(sp)[:, 0]
    inflow = np.stack([(-np.maximum(v1, 0) * fl[i] + np.minimum(v1, 0) * fr[i]) / dxs[i] for i in range(B)])
    nu = np.array([1.3 * OQ.nu_of(sp, fo[i]) for i in range(B)])
    g0 = 0.5 * (fo + fl)
    ctx = bz.Context(N=N, L=L, n_theta=nt, n_phi=nph, n_rho=nr)
    g, st = ctx.cell_fixed_point_ex(_T(fo), _T(inflow), _T(eps), nu=_T(nu), dxs=_T(dxs), g0=_T(g0), fixed_iters=2)
    g = g.cpu().numpy()
    s = bz.Context.decode_stats(st)
    checked = 0
    for i in range(B):
        Q = OQ.q_corrected(sp, fo[i], conserve="mass")
        M = discrete_maxwellian(sp, fo[i])
        P = OQ.penalty_split(Q, M, fo[i], nu[i])
        r = inflow[i] - P / eps[i]
        go, so = OC.solve(sp, r, nu[i], eps[i], dxs[i], g0[i], mode="pfp", fixed_iters=2)
        assert s["fallback"][i] == int(so.fallback)
        if so.fallback:
            continue  # the failure point of a step-1 Newton depends on rounding
        checked += 1
        assert np.abs(g[i] - go).max() < 1e-11 * np.abs(go).max(), i
    assert checked > 0


def test_strict_mode_reports_non_finite_results(bz):
    N, L = 8, 6.0
    sp = Spec(d=3, N=N, L=L, n_theta=2, n_phi=4, n_rho=2)
    ctx = bz.Context(N=N, L=L, n_theta=2, n_phi=4, n_rho=2)
    K = ctx.K
    # a slab of two instances, one with a non-finite cell
    f = torch.ones((6, K), dtype=torch.float64, device="cuda:0")
    f[4, 5] = float("nan")
    slab = bz.Slab(ctx, [dict(nx=3, eps=0.1), dict(nx=3, eps=0.1)], f, collision="bgk")
    res = slab.residual()
    assert np.isfinite(res[0]) and not np.isfinite(res[1])  # not strict: reported, no error
    ctx.set_strict(True)
    with pytest.raises(bz.BZNumericError):
        slab.residual()
    ctx.set_strict(False)
    # a cell call with a non-finite right-hand side in one cell
    fo, fl, fr, eps = synth.cell_inflow_batch(4, N, L, 1 / 16, seed=5)
    v1 = velocity_nodes(sp)[:, 0]
    r = (-np.maximum(v1, 0) * fl + np.minimum(v1, 0) * fr) * 16
    r[2, 3] = np.nan
    nu = np.array([OQ.nu_of(sp, fo[i]) for i in range(4)])
    g, st = ctx.cell_solve(_T(r), _T(nu), _T(eps), 1 / 16, _T(fo), fixed_iters=2)
    assert ctx.cell_check(st) == 1
    ctx.set_strict(True)
    with pytest.raises(bz.BZNumericError):
        ctx.cell_check(st)
    ctx.set_strict(False)
