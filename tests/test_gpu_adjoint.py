"""Adjoint of K FP64 steps (lbm_forward_record / lbm_backward) against the
oracle's exact forward-mode derivatives, and its own consistency checks."""
import numpy as np
import pytest

from oracle import Oracle, dual_forces, run_forces
from paper_1803_07822_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lbm():
    from paper_1803_07822_amd import lbm

    return lbm


def _case(nx=10, ny=7, nz=6, tau=0.7, seed=3):
    d = synth.gaussian_random_field(nx, nz, corr=2.5, max_abs=0.4, seed=seed)
    o = Oracle(nx, ny, nz, tau)
    o.set_wall_displacement(1, d)
    o.init_equilibrium(1 + synth.random_perturbation((nz, ny - 2, nx), 1e-3, seed + 1),
                       synth.random_perturbation((3, nz, ny - 2, nx), 1e-2, seed + 2))
    f0 = o.populations()
    return d, f0


def _gpu_grads(nx, ny, nz, tau, F, d, f0, K, N, W):
    lbm = _lbm()
    S = lbm.Solver(nx, ny, nz, tau, "fp64", adjoint_K=K, ckpt_every=N)
    S.set_body_force(F)
    S.set_wall_displacement(1, d)
    S.set_populations(f0)
    forces = S.forward_record(K).cpu().numpy()
    gd, gc, gf = S.backward(W, need_disp=True, need_chart=True, need_f0=True)
    return S, forces, gd.cpu().numpy(), gc.cpu().numpy(), gf.cpu().numpy()


def test_adjoint_matches_forward_mode_derivatives():
    nx, ny, nz, tau, K, N = 10, 7, 6, 0.7, 6, 2
    F = (1e-4, 0.0, 2e-5)
    d, f0 = _case(nx, ny, nz, tau)
    W = synth.random_perturbation((K, 3), 1.0, 17)
    S, forces, gd, gc, gf = _gpu_grads(nx, ny, nz, tau, F, d, f0, K, N, W)
    fo = run_forces(nx, ny, nz, tau, F, d, f0, K)
    assert np.abs(forces - fo).max() < 1e-12 * np.abs(fo).max()
    errs = []
    for r in range(4):
        dd = synth.random_unit(d.shape, 100 + r) if r != 1 else np.zeros(d.shape)
        df = synth.random_unit(f0.shape, 200 + r) * 1e-2 if r != 0 else np.zeros(f0.shape)
        _, dforces = dual_forces(nx, ny, nz, tau, F, d, dd, f0, df, K)
        exact = float((W * dforces).sum())
        adj = float((gd * dd).sum() + (gf * df).sum())
        errs.append(abs(adj - exact) / max(abs(exact), 1e-30))
        assert abs(exact) > 1e-12
    print("adjoint vs forward mode, relative errors:", errs)
    assert max(errs) < 1e-9, errs


def test_adjoint_chart_and_displacement_agree():
    """d enters only through chart_y = xi_y + (eta/H) d: <dL/dchart, dchart> = <dL/dd, dd>."""
    nx, ny, nz, tau, K, N = 10, 7, 6, 0.7, 4, 2
    d, f0 = _case(nx, ny, nz, tau, seed=5)
    W = synth.random_perturbation((K, 3), 1.0, 9)
    _, _, gd, gc, _ = _gpu_grads(nx, ny, nz, tau, (1e-4, 0, 0), d, f0, K, N, W)
    dd = synth.random_unit(d.shape, 31)
    dchart = synth.chart_from_displacement(nx, ny, nz, dd) - synth.identity_chart(nx, ny, nz)
    a = float((gc * dchart).sum())
    b = float((gd * dd).sum())
    assert abs(a - b) < 1e-12 * max(abs(a), abs(b))


@pytest.mark.parametrize("N", [1, 3, 6])
def test_adjoint_independent_of_checkpoint_interval(N):
    nx, ny, nz, tau, K = 10, 7, 6, 0.7, 6
    d, f0 = _case(nx, ny, nz, tau, seed=7)
    W = synth.random_perturbation((K, 3), 1.0, 23)
    _, _, gd_ref, _, gf_ref = _gpu_grads(nx, ny, nz, tau, (1e-4, 0, 0), d, f0, K, 2, W)
    _, _, gd, _, gf = _gpu_grads(nx, ny, nz, tau, (1e-4, 0, 0), d, f0, K, N, W)
    assert np.abs(gd - gd_ref).max() <= 1e-13 * np.abs(gd_ref).max()
    assert np.abs(gf - gf_ref).max() <= 1e-13 * np.abs(gf_ref).max()


def test_autograd_function():
    lbm = _lbm()
    nx, ny, nz, tau, K, N = 10, 7, 6, 0.7, 5, 2
    d, f0 = _case(nx, ny, nz, tau, seed=11)
    S = lbm.Solver(nx, ny, nz, tau, "fp64", adjoint_K=K, ckpt_every=N)
    S.set_body_force((1e-4, 0, 0))
    dt = torch.tensor(d, dtype=torch.float64, device=S.device, requires_grad=True)
    ft = torch.tensor(f0, dtype=torch.float64, device=S.device, requires_grad=True)
    forces = lbm.WallForceFn.apply(dt, ft, S, K)
    loss = forces[:, 0].sum()
    loss.backward()
    dd = synth.random_unit(d.shape, 41)
    _, dforces = dual_forces(nx, ny, nz, tau, (1e-4, 0, 0), d, dd, f0, np.zeros_like(f0), K)
    exact = dforces[:, 0].sum()
    adj = float((dt.grad.cpu().numpy() * dd).sum())
    assert abs(adj - exact) < 1e-9 * abs(exact)
    assert ft.grad is not None and torch.isfinite(ft.grad).all()

    # a second forward on the same solver replaces the recording: the first
    # graph's backward raises instead of returning the second's gradient
    f1 = lbm.WallForceFn.apply(dt, ft, S, K)
    f2 = lbm.WallForceFn.apply(dt, ft, S, K)
    with pytest.raises(RuntimeError, match="recorded another trajectory"):
        f1[:, 0].sum().backward()
    f2[:, 0].sum().backward()


def test_adjoint_rejects_fp32():
    lbm = _lbm()
    S = lbm.Solver(8, 6, 4, 0.8, "fp32")
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_reserve_adjoint(S.ctx, 4, 2)
    assert e.value.code == -6


def test_backward_refuses_a_wrongly_sized_gradient():
    """Solver.backward hands the library a [K, 3] dL/dF (the library reads K x 3
    doubles): a tensor with another number of entries is refused on the host."""
    lbm = _lbm()
    nx, ny, nz, tau, K, N = 8, 6, 4, 0.8, 4, 2
    S = lbm.Solver(nx, ny, nz, tau, "fp64", adjoint_K=K, ckpt_every=N)
    S.set_wall_displacement(1, np.zeros((nz, nx)))
    S.init_equilibrium()
    S.forward_record(K)
    for bad in (np.ones((K - 1, 3)), np.ones(3 * K + 1)):
        with pytest.raises(ValueError):
            S.backward(bad)
    gd, _, _ = S.backward(np.ones(3 * K))  # a flat array of the right size is taken as [K, 3]
    assert torch.isfinite(gd).all()


def test_backward_refuses_a_changed_setup():
    """A setter between forward_record and backward invalidates the recording
    (its checkpoints were taken with the old fields): ESTATE, until the next
    forward_record."""
    lbm = _lbm()
    nx, ny, nz, tau, K, N = 8, 6, 4, 0.8, 4, 2
    S = lbm.Solver(nx, ny, nz, tau, "fp64", adjoint_K=K, ckpt_every=N)
    S.set_wall_displacement(1, np.zeros((nz, nx)))
    S.init_equilibrium()
    W = np.ones((K, 3))
    changes = [
        lambda: S.set_body_force((1e-5, 0.0, 0.0)),
        lambda: S.set_wall_displacement(1, np.full((nz, nx), 0.1)),
        lambda: S.set_wall_velocity(0, np.full((nz, nx, 3), 1e-3)),
    ]
    for change in changes:
        S.forward_record(K)
        change()
        with pytest.raises(lbm.LBMError) as e:
            S.backward(W)
        assert e.value.code == -4
    S.forward_record(K)
    gd, _, gf = S.backward(W)
    assert torch.isfinite(gd).all() and torch.isfinite(gf).all()


def test_moving_wall_adjoint_matches_forward_mode_derivatives():
    """Both walls moving with seeded Cartesian velocities (halfway bounce-back
    with the moving-wall momentum term, and the gradient ghost 2 rho u_w - j,
    u_w = J^-1 v at the wall row): the gradients in the top-wall displacement
    and in f0 against the oracle's forward-mode derivatives of the same
    forces."""
    lbm = _lbm()
    nx, ny, nz, tau, K, N = 10, 7, 6, 0.7, 6, 2
    F = (1e-4, 0.0, 2e-5)
    d, f0 = _case(nx, ny, nz, tau, seed=5)
    vw = np.stack([synth.random_perturbation((nz, nx, 3), 1e-2, 31),
                   synth.random_perturbation((nz, nx, 3), 1e-2, 32)])
    W = synth.random_perturbation((K, 3), 1.0, 19)
    S = lbm.Solver(nx, ny, nz, tau, "fp64", adjoint_K=K, ckpt_every=N)
    S.set_body_force(F)
    S.set_wall_displacement(1, d)
    S.set_wall_velocity(0, vw[0])
    S.set_wall_velocity(1, vw[1])
    S.set_populations(f0)
    forces = S.forward_record(K).cpu().numpy()
    gd, gc, gf = S.backward(W, need_disp=True, need_chart=True, need_f0=True)
    gd, gc, gf = gd.cpu().numpy(), gc.cpu().numpy(), gf.cpu().numpy()
    # the chart gradient carries the same u_w term: <dL/dchart, dchart> = <dL/dd, dd>
    dd = synth.random_unit(d.shape, 33)
    dchart = synth.chart_from_displacement(nx, ny, nz, dd) - synth.identity_chart(nx, ny, nz)
    a, b = float((gc * dchart).sum()), float((gd * dd).sum())
    assert abs(a - b) < 1e-12 * max(abs(a), abs(b))
    fo = run_forces(nx, ny, nz, tau, F, d, f0, K, vwall=vw)
    f_rest = run_forces(nx, ny, nz, tau, F, d, f0, K)
    assert np.abs(fo - f_rest).max() > 1e-6 * np.abs(fo).max()
    assert np.abs(forces - fo).max() < 1e-12 * np.abs(fo).max()
    errs = []
    for r in range(3):
        dd = synth.random_unit(d.shape, 300 + r) if r != 1 else np.zeros(d.shape)
        df = synth.random_unit(f0.shape, 400 + r) * 1e-2 if r != 0 else np.zeros(f0.shape)
        _, dforces = dual_forces(nx, ny, nz, tau, F, d, dd, f0, df, K, vwall=vw)
        exact = float((W * dforces).sum())
        adj = float((gd * dd).sum() + (gf * df).sum())
        assert abs(exact) > 1e-12
        errs.append(abs(adj - exact) / abs(exact))
    print("moving-wall adjoint vs forward mode, relative errors:", errs)
    assert max(errs) < 1e-9, errs


def c4_setup():
    """The 128x64x64 adjoint workload: tau 0.7, body force 1e-6, top-wall
    displacement from a Gaussian random field (l = 8, max |d| = 0.05*64,
    seed 4) stored in FP32, initial state at rest."""
    w = synth.workload("c4_adjoint_128x64x64")
    d = w.disp().astype(np.float32).astype(np.float64)
    o = Oracle(w.nx, w.ny, w.nz, w.tau)  # the oracle only builds f0 here (no stepping)
    o.set_wall_displacement(1, d)
    o.init_equilibrium()
    return w, d, o.populations()


def test_c4_adjoint_against_central_differences():
    """Gradient of L = sum_{t=1..200} F_x(t) against FP64 central differences
    of the GPU forward (step 1e-6) on 16 seeded directions in d and 16 in f0."""
    lbm = _lbm()
    w, d, f0 = c4_setup()
    K, N = w.steps, w.extra["ckpt_every"]
    S = lbm.Solver(w.nx, w.ny, w.nz, w.tau, "fp64", adjoint_K=K, ckpt_every=N)
    S.set_body_force(w.force)

    def loss(dv, fv):
        S.set_wall_displacement(1, dv)
        S.set_populations(fv)
        return float(S.forward_record(K)[:, 0].sum().item())

    S.set_wall_displacement(1, d)
    S.set_populations(f0)
    S.forward_record(K)
    W = np.zeros((K, 3))
    W[:, 0] = 1.0
    gd, _, gf = S.backward(W)
    gd, gf = gd.cpu().numpy(), gf.cpu().numpy()
    # Directions have i.i.d. standard-normal entries (f0: scaled by the lattice
    # weights), so the step 1e-6 moves every entry by about 1e-6.
    eps = 1e-6
    wl = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)[:, None, None, None]
    errs_d, errs_f = [], []
    rng = np.random.Generator(np.random.PCG64(44))
    for r in range(16):
        v = rng.standard_normal(d.shape)
        fd = (loss(d + eps * v, f0) - loss(d - eps * v, f0)) / (2 * eps)
        errs_d.append(abs(fd - float((gd * v).sum())) / abs(fd))
        u = rng.standard_normal(f0.shape) * wl
        fdu = (loss(d, f0 + eps * u) - loss(d, f0 - eps * u)) / (2 * eps)
        errs_f.append(abs(fdu - float((gf * u).sum())) / abs(fdu))
    print(f"C4 FD check: max rel err d {max(errs_d):.2e}, f0 {max(errs_f):.2e}")
    assert max(errs_d) < 1e-3, errs_d
    assert max(errs_f) < 1e-3, errs_f


def test_backward_leaves_forward_final_state():
    """The reverse sweep rebuilds segments in its own trajectory storage: the
    context's state after lbm_backward is bit-for-bit the state
    lbm_forward_record ended with, and stepping on from it matches stepping
    on without the reverse sweep."""
    lbm = _lbm()
    nx, ny, nz, tau, K, N = 10, 7, 6, 0.7, 5, 2
    d, f0 = _case(nx, ny, nz, tau, seed=13)
    S = lbm.Solver(nx, ny, nz, tau, "fp64", adjoint_K=K, ckpt_every=N)
    S.set_body_force((1e-4, 0, 0))
    S.set_wall_displacement(1, d)
    S.set_populations(f0)
    S.forward_record(K)
    p_end, h_end = S.populations().cpu().numpy(), S.history().cpu().numpy()
    S.backward(synth.random_perturbation((K, 3), 1.0, 5))
    assert np.array_equal(S.populations().cpu().numpy(), p_end)
    assert np.array_equal(S.history().cpu().numpy(), h_end)
    S.step(3)
    o = Oracle(nx, ny, nz, tau)
    o.set_body_force((1e-4, 0, 0))
    o.set_wall_displacement(1, d)
    o.set_populations(f0)
    o.step(K + 3)
    fo = o.populations()
    assert np.abs(S.populations().cpu().numpy() - fo).max() < 1e-12 * np.abs(fo).max()
