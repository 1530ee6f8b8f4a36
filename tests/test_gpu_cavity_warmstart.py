"""The learned warm start in the 2D scans (bz_cavity_ws_attach) against the
oracle, through the C ABI: the transport part and the 2D feature rows, one SGS
iteration with a network whose output is the first visit's exact solution
(every candidate and choice compared one to one), convergence to the plain
state, and the argument checks.

A network with a zero last layer outputs exactly its last bias b3 (FP32
values, exact in both precisions), so candidates and choices compare one to
one with the FP64 oracle."""
import numpy as np
import pytest

from oracle import cavity as CV, cell as OC, collision as OQ, mlp as OM
from oracle.grid import Spec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SCAN_TOL = 1e-11  # as for the plain 2D scans
H = 16
WALLS = ((1.0, (0.0, 0.0)), (1.2, (0.0, 0.0)), (1.0, (0.0, 0.0)), (1.0, (0.4, 0.0)))


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_01910_amd as bz

    bz.load_library()
    return bz


def _setup(bz, N, nx, ny, collision, fixed, eps=0.2, order=1):
    sp = Spec(d=2, N=N, L=6.0, n_phi=8, n_rho=3)
    prob = CV.Cavity(spec=sp, nx=nx, ny=ny, eps=eps, walls=WALLS, collision=collision, fixed_inner=fixed,
                     order=order)
    f1 = CV.sgs_iteration(prob, CV.initial_state(prob))  # a state away from equilibrium
    ctx = bz.Context(N=N, L=6.0, n_phi=8, n_rho=3, d=2)
    return sp, prob, f1, ctx


def _first_visit_correction(prob, f):
    Q, M, nu = CV.all_collision(prob, f)
    P = OQ.penalty_split(Q, M, f, nu)
    T = CV.transport_part(prob, f)
    g, _ = OC.theta_solve(prob.spec, T[0, 0] - P[0, 0] / prob.eps, nu[0, 0], prob.eps, (prob.dx, prob.dy))
    return (g - M[0, 0]).astype(np.float32)


def _params(K, b3):
    p = np.zeros(OM.n_params(K + 5, H, K), dtype=np.float32)
    p[-K:] = b3
    return p


@pytest.mark.parametrize("N,order", [(8, 1), (8, 2), (32, 1)])
def test_inflow_and_features_match_oracle(bz, N, order):
    sp, prob, f1, ctx = _setup(bz, N, 3, 2, "binary", 2, order=order)
    fg = torch.from_numpy(f1.reshape(-1, sp.K).copy()).to("cuda:0").contiguous()
    cav = bz.Cavity(ctx, 3, 2, prob.eps, WALLS, fg, order=order)
    T = cav.inflow()
    theta, _, _ = ctx.maxwellian(fg)
    eps = torch.full((6,), prob.eps, dtype=torch.float64, device="cuda:0")
    X = ctx.features(T, theta, eps, prob.dx).cpu().numpy()
    Tref = CV.transport_part(prob, f1).reshape(-1, sp.K)
    scale = np.abs(Tref).max()
    assert np.abs(T.cpu().numpy() - Tref).max() < 1e-12 * scale
    for c in range(6):
        _, th = OC.discrete_maxwellian(sp, f1.reshape(-1, sp.K)[c], return_theta=True)
        xr = OM.features(sp, Tref[c], th, prob.eps, prob.dx)
        assert X.shape[1] == sp.K + 5
        assert np.abs(X[c] - xr).max() <= 1e-6 * np.abs(xr).max()  # FP32 rows


@pytest.mark.parametrize("N,collision", [(8, "binary"), (32, "binary"), (16, "bgk")])
def test_learned_cavity_scan_matches_oracle(bz, N, collision):
    print(f"learned cavity N={N} {collision}", flush=True)
    sp, prob, f1, ctx = _setup(bz, N, 3, 2, collision, 3)
    K = sp.K
    params = _params(K, _first_visit_correction(prob, f1))
    prob.warm = (params.astype(np.float64), K + 5, H, K, 1.0)
    prob.stats = {"inner": 0, "fallback": 0, "visits": 0, "learned": 0}
    f2 = CV.sgs_iteration(prob, f1)
    fg = torch.from_numpy(f1.reshape(-1, K).copy()).to("cuda:0").contiguous()
    cav = bz.Cavity(ctx, 3, 2, prob.eps, WALLS, fg, collision=collision, fixed_iters=3)
    mlp = bz.MLP(ctx, K + 5, H, K)
    mlp.set_params(params)
    mlp.set_output_scale(1.0)
    cav.attach_warmstart(mlp)
    res, st = cav.sweep(1)
    got = fg.cpu().numpy().reshape(f2.shape)
    err = np.abs(got - f2).max() / f2.max()
    ref = CV.outer_residual(prob, f2)
    print(f"  max rel diff {err:.3e}, residual {res:.6e} vs {ref:.6e}; learned starts {st['learned']} "
          f"(oracle {prob.stats['learned']}) of {st['visits']} visits", flush=True)
    assert err < SCAN_TOL
    assert abs(res - ref) < 1e-9 * ref
    assert st["learned"] == prob.stats["learned"] and 1 <= st["learned"] < st["visits"]


def test_learned_cavity_converges_to_the_plain_state(bz):
    N = 16
    sp = Spec(d=2, N=N, L=6.0, n_phi=8, n_rho=3)
    prob = CV.Cavity(spec=sp, nx=2, ny=2, eps=0.3, walls=WALLS, collision="bgk")
    f0 = CV.initial_state(prob)
    K = sp.K
    params = _params(K, _first_visit_correction(prob, f0))
    ctx = bz.Context(N=N, L=6.0, n_phi=8, n_rho=3, d=2)
    out, learned = [], []
    for attach in (False, True):
        fg = torch.from_numpy(f0.reshape(-1, K).copy()).to("cuda:0").contiguous()
        cav = bz.Cavity(ctx, 2, 2, 0.3, WALLS, fg, collision="bgk", tol=1e-12, max_iter=200)
        if attach:
            mlp = bz.MLP(ctx, K + 5, H, K)
            mlp.set_params(params)
            mlp.set_output_scale(1.0)
            cav.attach_warmstart(mlp)
        n_learned = 0
        for _ in range(300):
            res, st = cav.sweep(1)
            n_learned += st["learned"]
            if res < 1e-10:
                break
        print(f"attach={attach}: residual {res:.3e}, learned starts {n_learned}", flush=True)
        assert res < 1e-10
        out.append(fg.cpu().numpy())
        learned.append(n_learned)
    assert learned[0] == 0 and learned[1] >= 1
    assert np.abs(out[0] - out[1]).max() < 1e-8 * out[0].max()


def test_cavity_attach_arguments_are_checked(bz):
    ctx = bz.Context(N=8, L=6.0, n_phi=8, n_rho=3, d=2)
    K = ctx.K
    f = torch.ones((4, K), dtype=torch.float64, device="cuda:0")
    cav = bz.Cavity(ctx, 2, 2, 0.1, WALLS, f)
    with pytest.raises(bz.BZError):
        cav.attach_warmstart(bz.MLP(ctx, K + 6, H, K))  # the 2D input width is K + 5
    other = bz.Context(N=8, L=6.0, n_phi=8, n_rho=3, d=2)
    import ctypes

    wrong = bz.MLP(other, K + 5, H, K)
    assert ctx.lib.bz_cavity_ws_attach(cav.h, wrong.h) != 0  # a network of another context
    cav.attach_warmstart(bz.MLP(ctx, K + 5, H, K))
    cav.attach_warmstart(None)
    _ = ctypes
