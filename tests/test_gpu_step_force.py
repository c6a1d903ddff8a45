"""lbm_step_force (n steps, each giving the wall force of the state it steps
from) against lbm_wall_force followed by lbm_step, through the C-ABI.

On periodic grids without a plate the fused step forms the traction of
Sec. IV.A.2 from the stress its collision computes; the populations it leaves
must equal those of the plain step bit for bit, and the forces must agree
with the separate force kernel to rounding (FP64: 1e-13 of the summed stress
magnitude, FP32: 1e-6 of it, the two kernels forming T with different
rounding).  Grids with open ends or a plate, and the two-pass step, take the
separate kernels and must agree exactly."""
import numpy as np
import pytest

from paper_1803_07822_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lbm():
    from paper_1803_07822_amd import lbm

    return lbm


def _inlet(nz, H, U=0.02):
    eta = np.arange(H) + 0.5
    uin = np.zeros((nz, H, 3))
    uin[..., 0] = 4 * U * eta * (H - eta) / H**2
    return uin


def _solver(nx, ny, nz, precision, kind, seed, stream=None):
    lbm = _lbm()
    S = lbm.Solver(nx, ny, nz, 0.7, precision, stream=stream)
    H = ny - 2
    if kind == "open":
        S.set_open_x(_inlet(nz, H))
    if kind == "plate":
        S.set_plate(H // 2, nx // 4, nx // 2)
    S.set_body_force((1e-5, 0.0, 2e-6))
    S.set_wall_displacement(1, synth.gaussian_bump(nx, nz, A=0.3 * H / 8, x0=nx / 2, z0=nz / 3, sigma=3))
    if kind == "moving":
        for wall, v in ((0, (0.01, 0.0, -0.004)), (1, (-0.006, 0.002, 0.003))):
            vc = np.zeros((nz, nx, 3))
            vc[...] = v
            S.set_wall_velocity(wall, vc)
    if kind == "twopass":
        lbm.lbm_set_tuning(S.ctx, 0, 1, -1)
    S.init_equilibrium(None, synth.uniform_noise_velocity(nx, ny, nz, 1e-3, seed=seed))
    S.step(2)
    return S


def _run_pair(nx, ny, nz, precision, kind, wall, n, seed=3):
    lbm = _lbm()
    A = _solver(nx, ny, nz, precision, kind, seed)
    B = _solver(nx, ny, nz, precision, kind, seed)
    fa = torch.full((n, 3), float("nan"), dtype=torch.float64, device=A.device)
    fb = torch.full((n, 3), float("nan"), dtype=torch.float64, device=B.device)
    lbm.lbm_step_force(A.ctx, n, wall, fa)
    for t in range(n):
        lbm.lbm_wall_force(B.ctx, wall, fb[t])
        lbm.lbm_step(B.ctx, 1)
    A.sync()
    B.sync()
    pa, pb = A.populations().cpu().numpy(), B.populations().cpu().numpy()
    # scale of the summed stress: sqrt g |T^{iy}| is about 1/3 per column
    scale = nx * nz / 3.0
    out = fa.cpu().numpy(), fb.cpu().numpy(), pa, pb, scale
    del A, B
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(70, 12, 9), (150, 10, 44)])
@pytest.mark.parametrize("wall", [0, 1])
@pytest.mark.parametrize("kind", ["plain", "moving"])
def test_step_force_fused_matches_separate_kernels(precision, shape, wall, kind):
    fa, fb, pa, pb, scale = _run_pair(*shape, precision, kind, wall, n=5)
    assert np.isfinite(fa).all() and np.isfinite(fb).all()
    assert np.array_equal(pa, pb), "the fused force must not change the step"
    tol = 1e-13 if precision == "fp64" else 1e-6
    err = np.abs(fa - fb).max() / scale
    assert err < tol, (err, fa, fb)
    # the forces change from step to step (a real time series, not a copy)
    assert np.abs(np.diff(fb[:, 0])).max() > 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["open", "plate", "twopass"])
def test_step_force_fallback_is_exact(precision, kind):
    fa, fb, pa, pb, _ = _run_pair(40, 10, 8, precision, kind, 1, n=4)
    assert np.isfinite(fa).all()
    assert np.array_equal(pa, pb)
    assert np.array_equal(fa, fb)


def test_step_force_full_size_fp32():
    """The 256x128x128 bump channel (32 blocks hold the wall row per step)."""
    w = synth.workload("c2_bump_256x128x128")
    lbm = _lbm()
    S = [lbm.Solver(w.nx, w.ny, w.nz, w.tau, "fp32") for _ in range(2)]
    uc = synth.uniform_noise_velocity(w.nx, w.ny, w.nz, 1e-4, seed=2)
    for X in S:
        X.set_body_force(w.force)
        X.set_wall_displacement(lbm.LBM_WALL_YMAX, w.disp())
        X.init_equilibrium(None, uc)
    n = 4
    fa = torch.empty((n, 3), dtype=torch.float64, device=S[0].device)
    fb = torch.empty((n, 3), dtype=torch.float64, device=S[1].device)
    lbm.lbm_step_force(S[0].ctx, n, lbm.LBM_WALL_YMAX, fa)
    for t in range(n):
        lbm.lbm_wall_force(S[1].ctx, lbm.LBM_WALL_YMAX, fb[t])
        lbm.lbm_step(S[1].ctx, 1)
    for X in S:
        X.sync()
    fa, fb = fa.cpu().numpy(), fb.cpu().numpy()
    err = np.abs(fa - fb).max() / (w.nx * w.nz / 3.0)
    assert err < 1e-6, (err, fa, fb)
    assert np.array_equal(S[0].populations().cpu().numpy(), S[1].populations().cpu().numpy())


def test_step_force_argument_errors():
    lbm = _lbm()
    S = _solver(40, 10, 8, "fp64", "plain", 1)
    f = torch.zeros((2, 3), dtype=torch.float64, device=S.device)
    for args in ((-1, 1, f), (2, 2, f), (2, -1, f), (2, 1, None)):
        with pytest.raises(lbm.LBMError) as e:
            lbm.lbm_step_force(S.ctx, *args)
        assert e.value.code == -1  # LBM_EINVAL
    lbm.lbm_step_force(S.ctx, 0, 1, None)  # no steps, no output needed
    S.sync()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_step_force_graph_replays_match_eager(precision):
    """lbm_step_force captured on the context's stream and replayed: the fused
    kernel clears its own completion counter, so every replay matches the
    same call made eagerly on a second context, bit for bit."""
    lbm = _lbm()
    n = 4  # an even count: the buffer parity is back where it started
    side = torch.cuda.Stream()
    G = _solver(70, 12, 9, precision, "moving", 5, stream=side)
    E = _solver(70, 12, 9, precision, "moving", 5, stream=torch.cuda.Stream())
    fg = torch.zeros((n, 3), dtype=torch.float64, device=G.device)
    fe = torch.zeros((n, 3), dtype=torch.float64, device=G.device)
    # eager first (the launch shape is chosen on the first call), then capture
    lbm.lbm_step_force(G.ctx, n, 1, fg)
    lbm.lbm_step_force(E.ctx, n, 1, fe)
    G.sync()
    E.sync()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        lbm.lbm_step_force(G.ctx, n, 1, fg)
    torch.cuda.synchronize()
    for r in range(3):
        graph.replay()
        torch.cuda.synchronize()
        lbm.lbm_step_force(E.ctx, n, 1, fe)
        E.sync()
        G.sync()
        assert torch.equal(G.populations(), E.populations()), r
        assert torch.equal(fg, fe), r
