"""The learned warm start inside the slab scans (bz_ws_attach) against the oracle,
through the C ABI.

The network's output enters the visits only through the candidate
G = M[f_j] + scale * y.  A network with a zero last layer outputs exactly its
last bias b3 (FP32 values, exact in both precisions), so the candidates, the
residual-judged choice and every visit compare one to one with the FP64
oracle; b3 is the exact inner solution of one visit, so that visit takes the
candidate and the others keep their own state.  The BF16 products behind a
non-zero last layer are covered by the network's own GEMM tests."""
import numpy as np
import pytest

from oracle import cell as OC, mlp as OM, sweep as SW
from oracle.grid import Spec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SCAN_TOL = 1e-11  # as for the plain scans (see test_gpu_timed_sizes)
H = 16


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_01910_amd as bz

    bz.load_library()
    return bz


def _oracle_setup(N, inst, fixed):
    sp = Spec(d=3, N=N, L=8.0, n_theta=2, n_phi=4, n_rho=2)
    probs, f1 = [], []
    for d in inst:
        p = SW.Slab(spec=sp, nx=d["nx"], T_L=d.get("T_L", 1.0), T_R=d.get("T_R", 2.0), eps=d["eps"],
                    mass=d["mass"], collision="binary", fixed_inner=fixed)
        f = SW.sgs_iteration(p, SW.initial_state(p, T=1.5))  # a state away from equilibrium
        probs.append(p)
        f1.append(f)
    return sp, probs, f1


def _first_visit_candidate(prob, f):
    Q, M, nu = SW.all_collision(prob, f)
    P = SW.penalty_split(Q, M, f, nu)
    T = SW.transport_part(prob, f)
    g, _ = OC.theta_solve(prob.spec, T[0] - P[0] / prob.eps, nu[0], prob.eps, prob.dx)
    return (g - M[0]).astype(np.float32)


def _params(K, b3):
    p = np.zeros(OM.n_params(K + 6, H, K), dtype=np.float32)
    p[-K:] = b3
    return p


@pytest.mark.parametrize("N", [16, 32])
def test_learned_scan_matches_oracle(bz, N):
    inst = [dict(nx=3, eps=0.1, mass=1.0), dict(nx=2, eps=0.02, T_L=1.2, T_R=1.6, mass=0.9)]
    print(f"learned scan N={N}", flush=True)
    sp, probs, f1 = _oracle_setup(N, inst, fixed=3)
    K = sp.K
    b3 = _first_visit_candidate(probs[0], f1[0])
    params = _params(K, b3)
    learned_ref = 0
    f2 = []
    for p, f in zip(probs, f1):
        p.warm = (params.astype(np.float64), K + 6, H, K, 1.0)
        p.stats = {"inner": 0, "fallback": 0, "visits": 0, "learned": 0}
        f2.append(SW.sgs_iteration(p, f))
        learned_ref += p.stats["learned"]
    ctx = bz.Context(N=N, L=8.0, n_theta=2, n_phi=4, n_rho=2)
    fg = torch.from_numpy(np.concatenate(f1)).to("cuda:0").contiguous()
    slab = bz.Slab(ctx, inst, fg, fixed_iters=3)
    mlp = bz.MLP(ctx, K + 6, H, K)
    mlp.set_params(params)
    mlp.set_output_scale(1.0)
    slab.attach_warmstart(mlp)
    res, st = slab.sweep(1)
    got = fg.cpu().numpy()
    o = 0
    for i, d in enumerate(inst):
        err = np.abs(got[o:o + d["nx"]] - f2[i]).max() / f2[i].max()
        ref = SW.outer_residual(probs[i], f2[i])
        print(f"  instance {i}: max rel diff {err:.3e}, residual {res[i]:.6e} vs {ref:.6e}", flush=True)
        assert err < SCAN_TOL
        assert abs(res[i] - ref) < 1e-9 * ref
        o += d["nx"]
    print(f"  learned starts taken: {st['learned']} (oracle {learned_ref}) of {st['visits']} visits", flush=True)
    assert st["learned"] == learned_ref and 1 <= learned_ref < st["visits"]


def test_learned_scan_converges_to_the_plain_state(bz):
    # tolerance-based inner solves (1e-8), BGK collision (which converges in a
    # few dozen scans on 16^3): with the network attached the scans reach the
    # state the plain scans reach; the network's output is the exact solution of
    # the first visit from the initial state, so it is taken at least there
    N = 16
    sp = Spec(d=3, N=N, L=8.0, n_theta=2, n_phi=4, n_rho=2)
    inst = [dict(nx=4, eps=0.1, mass=1.0)]
    prob = SW.Slab(spec=sp, nx=4, eps=0.1, mass=1.0, collision="bgk")
    f0 = SW.initial_state(prob, T=1.5)
    K = sp.K
    params = _params(K, _first_visit_candidate(prob, f0))
    ctx = bz.Context(N=N, L=8.0, n_theta=2, n_phi=4, n_rho=2)
    out, learned = [], []
    for attach in (False, True):
        fg = torch.from_numpy(f0.copy()).to("cuda:0").contiguous()
        slab = bz.Slab(ctx, inst, fg, collision="bgk")
        if attach:
            mlp = bz.MLP(ctx, K + 6, H, K)
            mlp.set_params(params)
            mlp.set_output_scale(1.0)
            slab.attach_warmstart(mlp)
        n_learned = 0
        for _ in range(200):
            res, st = slab.sweep(1)
            n_learned += st["learned"]
            if res[0] < 1e-9:
                break
        print(f"attach={attach}: residual {res[0]:.3e}, learned starts {n_learned}", flush=True)
        assert res[0] < 1e-9
        out.append(fg.cpu().numpy())
        learned.append(n_learned)
    assert learned[0] == 0 and learned[1] >= 1
    assert np.abs(out[0] - out[1]).max() < 1e-8 * out[0].max()


def test_attach_arguments_and_capture_are_checked(bz):
    N = 8
    ctx = bz.Context(N=N, L=6.0, n_theta=2, n_phi=4, n_rho=2)
    K = ctx.K
    fg = torch.ones((2, K), dtype=torch.float64, device="cuda:0")
    slab = bz.Slab(ctx, [dict(nx=2, eps=0.1)], fg)
    with pytest.raises(bz.BZError):
        slab.attach_warmstart(bz.MLP(ctx, K, H, K))  # input width must be K + 6
    other = bz.Context(N=N, L=6.0, n_theta=2, n_phi=4, n_rho=2)
    with pytest.raises(bz.BZError):
        slab.attach_warmstart(bz.MLP(other, K + 6, H, K))  # another context
    slab.attach_warmstart(bz.MLP(ctx, K + 6, H, K))
    with pytest.raises(bz.BZError):
        slab.capture(1)
    slab.attach_warmstart(None)
    g = slab.capture(1)
    g.close()
