"""GPU parity: the HIP library (through its C-ABI) against the FP64 oracle on
the same seeded inputs.

FP64 form: element-wise agreement to rounding (the two differ only in the
order of floating-point operations).  FP32 deviation form: agreement within a
bound derived from FP32 rounding of the deviation variables.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_1803_07822_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def _lbm():
    from paper_1803_07822_amd import lbm

    return lbm


def _np(t):
    return t.detach().cpu().numpy()


def dev_err(a, b, ref):
    """max |a - b| relative to the largest deviation of ref from the weights."""
    scale = np.abs(ref - W.reshape((19,) + (1,) * (ref.ndim - 1))).max()
    return np.abs(a - b).max() / scale


def make_pair(nx, ny, nz, tau, precision="fp64", chart=None, disp=None, F=(0, 0, 0), vwall=None):
    lbm = _lbm()
    S = lbm.Solver(nx, ny, nz, tau, precision)
    O = Oracle(nx, ny, nz, tau)
    S.set_body_force(F)
    O.set_body_force(F)
    if vwall is not None:
        for w in (0, 1):
            if vwall[w] is not None:
                S.set_wall_velocity(w, vwall[w])
                O.set_wall_velocity(w, vwall[w])
    if chart is not None:
        S.set_metric(chart)
        O.set_metric(chart)
    else:
        S.set_wall_displacement(1, disp)
        O.set_wall_displacement(1, disp)
    return S, O


GEO_CASES = {
    "bump3_70x12x9": lambda: (70, 12, 9, synth.bump3_chart(70, 12, 9, 0.08), None),
    "disp_gauss_33x10x17": lambda: (33, 10, 17, None, synth.gaussian_bump(33, 17, A=1.5, x0=16, z0=8, sigma=3)),
    "identity_5x4x3": lambda: (5, 4, 3, synth.identity_chart(5, 4, 3), None),
}


@pytest.mark.parametrize("case", sorted(GEO_CASES))
def test_geometry_parity_fp64(case):
    nx, ny, nz, chart, disp = GEO_CASES[case]()
    S, O = make_pair(nx, ny, nz, 0.8, chart=chart, disp=disp, F=(1e-5, -3e-6, 2e-6))
    geo, jac = S.geometry()
    og, oj = O.geometry(), O.jacobian()
    assert np.abs(_np(jac) - oj).max() < 1e-13
    g = _np(geo)
    # sqrt g and g^ij are O(1): absolute agreement to rounding
    assert np.abs(g[:7] - og[:7]).max() < 1e-13
    # Christoffel symbols and F^i: relative to the largest entry of the field group
    gam_scale = np.abs(og[7:25]).max()
    assert np.abs(g[7:25] - og[7:25]).max() <= 1e-11 * gam_scale + 1e-16
    f_scale = np.abs(og[25:]).max()
    assert np.abs(g[25:] - og[25:]).max() <= 1e-13 * f_scale


def _random_state(O, nz, H, nx, seed):
    O.init_equilibrium(1 + synth.random_perturbation((nz, H, nx), 2e-3, seed),
                       synth.random_perturbation((3, nz, H, nx), 1e-2, seed + 1))
    f = O.populations() + synth.random_perturbation((19, nz, H, nx), 1e-4, seed + 2) * W[:, None, None, None]
    return f


@pytest.mark.parametrize("shape,variant,zc,stage", [((70, 12, 9), 0, 0, -1), ((64, 8, 4), 0, 0, -1),
                                                    ((7, 5, 3), 0, 0, -1), ((70, 12, 9), 1, 0, -1),
                                                    ((70, 12, 9), 0, 3, -1), ((33, 9, 11), 0, 5, -1),
                                                    ((70, 12, 9), 0, 4, 1), ((1, 4, 1), 0, 0, -1),
                                                    ((1, 6, 5), 1, 0, -1), ((3, 4, 2), 0, 1, -1),
                                                    ((65, 4, 1), 0, 0, -1), ((140, 7, 9), 0, 0, -1),
                                                    ((300, 5, 6), 0, 4, -1), ((1, 4, 1), 1, 0, -1)])
def test_step_parity_fp64(shape, variant, zc, stage):
    """Curved chart, body force, moving walls, non-equilibrium start: the GPU
    state matches the oracle population by population after 1 and 12 steps;
    history, moments and wall forces too.  Shapes span several 64x4 tiles with
    ragged edges in x and y and several z chunks, in the fused and the
    two-pass step, and the degenerate grids: a single column
    (nx = nz = 1, every neighbour is the node itself), the thinnest channel
    (two fluid layers, both next to a wall) and a single z-plane."""
    nx, ny, nz = shape
    H = ny - 2
    vt = np.zeros((nz, nx, 3))
    vt[..., 0], vt[..., 2] = 0.01, -0.003
    vb = np.zeros((nz, nx, 3))
    vb[..., 1] = 0.0  # normal velocity stays zero at a wall at rest in y
    vb[..., 2] = 0.004
    S, O = make_pair(nx, ny, nz, 0.7, chart=synth.bump3_chart(nx, ny, nz, 0.06), F=(2e-5, 0, 1e-5), vwall=(vb, vt))
    _lbm().lbm_set_tuning(S.ctx, zc, variant, stage)
    f0 = _random_state(O, nz, H, nx, 21)
    O.set_populations(f0)
    S.set_populations(f0)
    assert dev_err(_np(S.populations()), O.populations(), f0) < 1e-13
    assert np.abs(_np(S.history()) - O.history()).max() < 1e-14
    for n in (1, 11):
        O.step(n)
        S.step(n)
        fo = O.populations()
        assert dev_err(_np(S.populations()), fo, fo) < 1e-12, n
        assert np.abs(_np(S.history()) - O.history()).max() < 1e-13
        r, u = S.moments(cartesian=True)
        ro, uo = O.moments(cartesian=True)
        assert np.abs(_np(r) - ro).max() < 1e-13
        assert np.abs(_np(u) - uo).max() < 1e-13
        for wall in (0, 1):
            t, pn = S.wall_force(wall, per_node=True)
            to, pno = O.wall_force(wall, per_node=True)
            assert np.abs(_np(pn) - pno).max() < 1e-13
            assert np.abs(_np(t) - to).max() < 1e-12 * max(1.0, np.abs(to).max())


def test_init_equilibrium_parity_fp64():
    nx, ny, nz = 40, 9, 6
    d = synth.gaussian_bump(nx, nz, A=1.0, x0=20, z0=3, sigma=3)
    S, O = make_pair(nx, ny, nz, 0.9, disp=d, F=(1e-5, 0, 0))
    rho = 1 + synth.random_perturbation((nz, ny - 2, nx), 1e-3, 5)
    uc = synth.random_perturbation((3, nz, ny - 2, nx), 1e-2, 6)
    S.init_equilibrium(rho, uc)
    O.init_equilibrium(rho, uc)
    fo = O.populations()
    assert dev_err(_np(S.populations()), fo, fo) < 1e-13
    assert np.abs(_np(S.history()) - O.history()).max() < 1e-14


def test_reprojection_parity_fp64():
    nx, ny, nz = 48, 10, 12
    H = ny - 2
    d1 = synth.gaussian_bump(nx, nz, A=1.2, x0=24, z0=6, sigma=4)
    d2 = 0.7 * d1 + 0.3 * np.sin(2 * np.pi * np.arange(nx) / nx)[None, :]
    v = np.zeros((nz, nx, 3))
    v[..., 1] = 0.002 * np.cos(2 * np.pi * np.arange(nx) / nx)[None, :]
    S, O = make_pair(nx, ny, nz, 0.75, disp=d1, F=(1e-5, 0, 0), vwall=(None, v))
    f0 = _random_state(O, nz, H, nx, 31)
    O.set_populations(f0)
    S.set_populations(f0)
    O.step(3)
    S.step(3)
    O.set_wall_displacement(1, d2, reproject=True)
    S.set_wall_displacement(1, d2, reproject=True)
    fo = O.populations()
    assert dev_err(_np(S.populations()), fo, fo) < 1e-12
    assert np.abs(_np(S.history()) - O.history()).max() < 1e-13
    O.step(4)
    S.step(4)
    fo = O.populations()
    assert dev_err(_np(S.populations()), fo, fo) < 1e-12
    # generic chart entry point with re-projection
    ch = synth.bump3_chart(nx, ny, nz, 0.05)
    O.set_metric(ch, reproject=True)
    S.set_metric(ch, reproject=True)
    fo = O.populations()
    assert dev_err(_np(S.populations()), fo, fo) < 1e-12
    # back to a wall-displacement chart: the old chart moves x and z, so the
    # search for psi must be the three-dimensional one
    O.set_wall_displacement(1, d1, reproject=True)
    S.set_wall_displacement(1, d1, reproject=True)
    fo = O.populations()
    assert dev_err(_np(S.populations()), fo, fo) < 1e-12
    assert np.abs(_np(S.history()) - O.history()).max() < 1e-13
    # and on from there between two wall charts (one-dimensional search)
    O.set_wall_displacement(1, d2, reproject=True)
    S.set_wall_displacement(1, d2, reproject=True)
    fo = O.populations()
    assert dev_err(_np(S.populations()), fo, fo) < 1e-12


def test_reprojection_parity_fp32():
    """The FP32 deviation form through a wall re-projection, a generic chart
    re-projection and steps after each: the moment fields of the
    re-projection are stored in FP32 (deviations from rest) and the new state
    is rounded to FP32, so populations and history agree with the FP64 oracle
    to the FP32 rounding of the deviation variables (about 1e-7 of their
    scale per operation; bound 1e-5 over the ~10 roundings on the path)."""
    nx, ny, nz = 48, 10, 12
    H = ny - 2
    d1 = synth.gaussian_bump(nx, nz, A=1.2, x0=24, z0=6, sigma=4)
    d2 = 0.7 * d1 + 0.3 * np.sin(2 * np.pi * np.arange(nx) / nx)[None, :]
    v = np.zeros((nz, nx, 3))
    v[..., 1] = 0.002 * np.cos(2 * np.pi * np.arange(nx) / nx)[None, :]
    S, O = make_pair(nx, ny, nz, 0.75, precision="fp32", disp=d1, F=(1e-5, 0, 0), vwall=(None, v))
    f0 = _random_state(O, nz, H, nx, 31)
    O.set_populations(f0)
    S.set_populations(f0)
    O.step(3)
    S.step(3)

    def check(tag):
        fo, ho = O.populations(), O.history()
        ef = dev_err(_np(S.populations()), fo, fo)
        eh = np.abs(_np(S.history()) - ho).max() / np.abs(ho).max()
        print(f"fp32 re-projection {tag}: populations {ef:.2e}, history {eh:.2e}", flush=True)
        assert ef < 1e-5, (tag, ef)
        assert eh < 1e-5, (tag, eh)

    O.set_wall_displacement(1, d2, reproject=True)
    S.set_wall_displacement(1, d2, reproject=True)
    check("wall")
    O.step(4)
    S.step(4)
    check("wall + 4 steps")
    ch = synth.bump3_chart(nx, ny, nz, 0.05)
    O.set_metric(ch, reproject=True)
    S.set_metric(ch, reproject=True)
    check("chart")
    O.step(4)
    S.step(4)
    check("chart + 4 steps")
    O.set_wall_displacement(1, d1, reproject=True)
    S.set_wall_displacement(1, d1, reproject=True)
    check("chart to wall")
    r, u = S.moments(cartesian=True)
    ro, uo = O.moments(cartesian=True)
    assert np.abs(_np(r) - ro).max() < 2e-6
    assert np.abs(_np(u) - uo).max() / np.abs(uo).max() < 1e-4


def test_config1_channel_parity_fp64():
    """The 32x16x16 sheared channel, tau 0.8, F 1e-6, 2000 steps."""
    w = synth.workload("c1_shear_32x16x16")
    S, O = make_pair(w.nx, w.ny, w.nz, w.tau, disp=w.disp(), F=w.force)
    S.init_equilibrium()
    O.init_equilibrium()
    S.step(w.steps)
    O.step(w.steps)
    r, u = S.moments(cartesian=True)
    ro, uo = O.moments(cartesian=True)
    eu = np.abs(_np(u) - uo).max() / np.abs(uo).max()
    # rho carries the rounding of 2000 mass updates (~1e-16 each, same sign on
    # all nodes): bound 2000 * 2.5e-16
    er = np.abs(_np(r) - ro).max()
    fo = O.populations()
    ef = dev_err(_np(S.populations()), fo, fo)
    assert eu < 1e-10, eu
    assert er < 5e-13, er
    assert ef < 1e-10, ef


@pytest.mark.parametrize("shape,variant,zc,stage", [((70, 12, 9), 0, 0, -1), ((32, 16, 16), 0, 0, -1),
                                                    ((33, 9, 11), 0, 5, 1), ((70, 12, 9), 0, 4, 1),
                                                    ((70, 12, 9), 1, 0, -1), ((70, 12, 9), 0, 0, 0),
                                                    ((70, 12, 9), 0, 3, 0), ((33, 9, 11), 0, 4, 0),
                                                    ((7, 5, 3), 0, 0, 1), ((7, 5, 3), 0, 0, 0),
                                                    ((140, 7, 9), 0, 0, 1), ((300, 5, 6), 0, 4, 1),
                                                    ((140, 7, 9), 0, 3, 0)])
def test_step_parity_fp32(shape, variant, zc, stage):
    """FP32 deviation storage and arithmetic against the FP64 oracle: errors in
    rho, u and wall force stay at the FP32 rounding level of the deviation
    variables.  Covers the fused step with both stagings of the pulled
    populations (re-read, registers) and the two-pass step, ragged tiles and
    z chunks, and a moving top wall."""
    nx, ny, nz = shape
    H = ny - 2
    vt = np.zeros((nz, nx, 3))
    vt[..., 0] = 0.01
    S, O = make_pair(nx, ny, nz, 0.7, precision="fp32", chart=synth.bump3_chart(nx, ny, nz, 0.06), F=(1e-5, 0, 0),
                     vwall=(None, vt))
    _lbm().lbm_set_tuning(S.ctx, zc, variant, stage)
    f0 = _random_state(O, nz, H, nx, 41)
    O.set_populations(f0)
    S.set_populations(f0)
    O.step(50)
    S.step(50)
    r, u = S.moments(cartesian=True)
    ro, uo = O.moments(cartesian=True)
    er = np.abs(_np(r) - ro).max()
    eu = np.abs(_np(u) - uo).max() / np.abs(uo).max()
    t = _np(S.wall_force(1))
    to = O.wall_force(1)
    ef = np.abs(t - to).max() / np.abs(to).max()
    print(f"fp32 {shape}: max|drho| {er:.2e}, max|du|/max|u| {eu:.2e}, wall force rel {ef:.2e}")
    assert er < 2e-6
    assert eu < 1e-4
    assert ef < 1e-5


def test_instability_guard_reports_nonfinite_state():
    lbm = _lbm()
    nx, ny, nz = 16, 8, 4
    S = lbm.Solver(nx, ny, nz, 0.8)
    S.set_wall_displacement(1, np.zeros((nz, nx)))
    f = np.tile(W[:, None, None, None], (1, nz, ny - 2, nx))
    f[3, 1, 2, 5] = np.nan
    S.set_populations(f)
    S.step(2)
    with pytest.raises(lbm.LBMError) as e:
        S.sync()
    assert e.value.code == -5
    with pytest.raises(lbm.LBMError) as e:  # sticky
        S.step(1)
    assert e.value.code == -5


def test_call_order_and_argument_errors():
    lbm = _lbm()
    S = lbm.Solver(8, 6, 4, 0.8)
    with pytest.raises(lbm.LBMError) as e:
        S.step(1)
    assert e.value.code == -4
    with pytest.raises(lbm.LBMError) as e:
        S.init_equilibrium()
    assert e.value.code == -4
    S.set_wall_displacement(1, np.zeros((4, 8)))
    with pytest.raises(lbm.LBMError) as e:
        S.set_wall_displacement(1, np.zeros((4, 8)), reproject=True)
    assert e.value.code == -4
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_wall_force(S.ctx, 2, torch.zeros(3, dtype=torch.float64, device=S.device))
    assert e.value.code == -1
    S.init_equilibrium()
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_step(S.ctx, -1)
    assert e.value.code == -1
    S.step(3)
    S.sync()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_tuning_round_trip(precision):
    """lbm_set_tuning / lbm_get_tuning: explicit shapes come back as set, the
    automatic z chunk resolves to a plane count in 1..nz, FP64 never runs the
    register staging, and bad arguments are refused."""
    lbm = _lbm()
    nx, ny, nz = 130, 20, 40
    S = lbm.Solver(nx, ny, nz, 0.8, precision)
    z, v, st = lbm.lbm_get_tuning(S.ctx)
    assert 1 <= z <= nz and v == 0 and st == (1 if precision == "fp32" else 0)
    lbm.lbm_set_tuning(S.ctx, 7, 0, 0)
    assert lbm.lbm_get_tuning(S.ctx) == (7, 0, 0)
    lbm.lbm_set_tuning(S.ctx, 500, 0, 1)
    assert lbm.lbm_get_tuning(S.ctx) == (nz, 0, 1 if precision == "fp32" else 0)
    lbm.lbm_set_tuning(S.ctx, 0, 1, -1)
    assert lbm.lbm_get_tuning(S.ctx)[:2] == (0, 1)
    for bad in ((-1, 0, -1), (0, 2, -1), (0, 5, -1), (0, -1, -1), (0, 0, 2), (0, 0, -2)):
        with pytest.raises(lbm.LBMError) as e:
            lbm.lbm_set_tuning(S.ctx, *bad)
        assert e.value.code == -1


@pytest.mark.parametrize("chart", ["affine_shear", "diagonal_metric", "sin_shear"])
def test_curved_poiseuille_steady_state(chart):
    """Steady Poiseuille flow in charts of the flat channel (H = 16, 5190
    steps): the GPU's FP64 steady state matches the oracle's, and its FP32
    Cartesian profile matches the FP64 one to FP32 rounding."""
    H, tau, F = 16, 0.8, 1e-6
    nx, ny, nz = 2, H + 2, 1
    if chart == "affine_shear":
        ch = synth.identity_chart(nx, ny, nz)
        ch[0] += 0.05 * (ch[1] - 0.5)
    elif chart == "diagonal_metric":
        ch = synth.diagonal_metric_chart(nx, ny, nz, 0.1 * (H / 8.0) ** 2)
    else:
        ch = synth.shear_chart(nx, ny, nz, 0.05)
    nu = (tau - 0.5) / 3
    steps = int(20 / (nu * (np.pi / H) ** 2))
    O = Oracle(nx, ny, nz, tau)
    O.set_body_force((F, 0, 0))
    O.set_metric(ch)
    O.init_equilibrium()
    O.step(steps)
    _, uo = O.moments(cartesian=True)
    out = {}
    for precision in ("fp64", "fp32"):
        S = _lbm().Solver(nx, ny, nz, tau, precision)
        S.set_body_force((F, 0, 0))
        S.set_metric(ch)
        S.init_equilibrium()
        S.step(steps)
        out[precision] = _np(S.moments(cartesian=True)[1])
    scale = np.abs(uo).max()
    assert np.abs(out["fp64"] - uo).max() < 1e-10 * scale
    assert np.abs(out["fp32"] - out["fp64"]).max() < 1e-3 * scale


@pytest.mark.parametrize("precision,variant", [("fp64", 0), ("fp64", 1), ("fp32", 0)])
def test_wall_force_momentum_exchange_parity(precision, variant):
    """Momentum-exchange force (diagnostic, walls at rest) of both walls in a
    curved chart after a non-equilibrium start and 1, 7 steps, per column,
    against the oracle; a wall given a velocity is refused, and so is an
    unknown method."""
    lbm = _lbm()
    nx, ny, nz = 70, 12, 9
    H = ny - 2
    S, O = make_pair(nx, ny, nz, 0.7, precision=precision, chart=synth.bump3_chart(nx, ny, nz, 0.06),
                     F=(2e-5, -1e-6, 1e-5))
    lbm.lbm_set_tuning(S.ctx, 0, variant, -1)
    f0 = _random_state(O, nz, H, nx, 51)
    O.set_populations(f0)
    S.set_populations(f0)
    for n in (1, 6):
        O.step(n)
        S.step(n)
        for wall in (0, 1):
            t, pn = S.wall_force(wall, per_node=True, method=lbm.LBM_FORCE_MEM)
            to, pno = O.wall_force_mem(wall, per_node=True)
            scale = np.abs(pno).max()
            tol = 1e-13 if precision == "fp64" else 2e-6
            assert np.abs(_np(pn) - pno).max() < tol * scale, (wall, n)
            assert np.abs(_np(t) - to).max() < tol * np.abs(to).max() * 10
    tot = torch.zeros(3, dtype=torch.float64, device=S.device)
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_wall_force(S.ctx, 1, tot, None, 2)
    assert e.value.code == -1
    S.set_wall_velocity(1, np.zeros((nz, nx, 3)))
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_wall_force(S.ctx, 1, tot, None, lbm.LBM_FORCE_MEM)
    assert e.value.code == -6


@pytest.mark.parametrize("case", ["fused", "two_pass", "open_fused"])
def test_step_profiled_matches_plain_steps(case):
    """lbm_step_profiled runs the same step as lbm_step (states equal bit for
    bit) and times its kernels in two slots: the fused kernel (second slot
    empty; with open ends, the end-column passes there) or the two passes."""
    lbm = _lbm()
    nx, ny, nz = 70, 12, 9
    H = ny - 2
    ctxs = []
    for _ in range(2):
        S = lbm.Solver(nx, ny, nz, 0.7, "fp32")
        S.set_body_force((1e-5, 0, 0))
        if case == "open_fused":
            S.set_open_x(synth.parabolic_inlet(nz, H, 0.04))
        S.set_metric(synth.bump3_chart(nx, ny, nz, 0.05))
        lbm.lbm_set_tuning(S.ctx, 0, 1 if case == "two_pass" else 0, -1)
        S.init_equilibrium(None, synth.random_perturbation((3, nz, H, nx), 1e-2, 5))
        ctxs.append(S)
    A, B = ctxs
    ms = lbm.lbm_step_profiled(A.ctx, 3)
    B.step(3)
    B.sync()
    assert torch.equal(A.populations(), B.populations())
    assert torch.equal(A.history(), B.history())
    print(case, "slots (ms):", ms, flush=True)
    assert ms[0] > 0 and ms[2] == 0 and ms[3] == 0
    if case == "fused":
        assert ms[1] < 0.5 * ms[0]  # two events back to back
    else:
        assert ms[1] > 0
    for bad in ((0, 4), (1, 1)):
        with pytest.raises(lbm.LBMError) as e:
            lbm.lbm_step_profiled(A.ctx, *bad)
        assert e.value.code == -1
