"""Launch-bound loops replayed as HIP graphs: a sequence of library calls on
the context's own stream (steps, plate shape with re-projection, plate
velocity, plate force; or a wall alternately moved and cleared) captured
once and replayed.  Every replay is checked
against the same calls made eagerly on a second context, with eager work and
synchronisations between the replays; the graph holds kernels and
device-to-device copies only (no memsets)."""
import numpy as np
import pytest

from paper_1803_07822_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lbm():
    from paper_1803_07822_amd import lbm

    return lbm


def _flag_solver(precision, stream, variant=None):
    lbm = _lbm()
    nx, ny, nz, tau = 64, 18, 1, 0.7
    H = ny - 2
    S = lbm.Solver(nx, ny, nz, tau, precision, stream=stream)
    if variant is not None:  # else the automatic choice (the two-pass step on this small open grid)
        lbm.lbm_set_tuning(S.ctx, 0, variant, -1)
    S.set_open_x(synth.parabolic_inlet(nz, H, 0.04))
    S.set_plate(8, 12, 30)
    S.set_wall_displacement(1, np.zeros((nz, nx)))
    uc = np.zeros((3, nz, H, nx))
    uc[0] = synth.parabolic_inlet(nz, H, 0.04)[..., 0][:, :, None]
    S.init_equilibrium(None, uc)
    return S


@pytest.mark.parametrize("precision,variant", [("fp64", None), ("fp32", None), ("fp32", 0), ("fp64", 0)])
def test_flag_loop_graph_replays_match_eager(precision, variant):
    """variant None: the automatic step (two-pass here); 0: the fused step
    with its end-column passes."""
    lbm = _lbm()
    nx, nz, steps = 64, 1, 4  # an even count: the context's buffer parity is back where it started
    shapes = [synth.flapping_plate(nx, nz, 12, 30, A=0.3, omega=2 * np.pi / 200, t=float(t)) for t in range(steps)]
    side = torch.cuda.Stream()
    G = _flag_solver(precision, side, variant)  # replayed
    E = _flag_solver(precision, torch.cuda.Stream(), variant)  # eager
    dev = [(torch.as_tensor(d, device=G.device), torch.as_tensor(v, device=G.device)) for d, v in shapes]
    fg = torch.zeros((steps, 3), dtype=torch.float64, device=G.device)
    fe = torch.zeros((steps, 3), dtype=torch.float64, device=G.device)

    def calls(S, force):
        for t in range(steps):
            lbm.lbm_step(S.ctx, 1)
            lbm.lbm_set_plate_displacement(S.ctx, dev[t][0], 1)
            lbm.lbm_set_plate_velocity(S.ctx, dev[t][1])
            lbm.lbm_plate_force(S.ctx, force[t])

    # one eager pass on each first (the step kernel's launch shape is chosen
    # on its first call, outside the capture), then capture
    calls(G, fg)
    calls(E, fe)
    G.sync()
    E.sync()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        calls(G, fg)
    torch.cuda.synchronize()
    for r in range(3):
        graph.replay()
        torch.cuda.synchronize()
        calls(E, fe)
        E.sync()
        G.sync()
        pg, pe = G.populations(), E.populations()
        assert torch.equal(pg, pe), (r, float((pg - pe).abs().max()))
        assert torch.equal(fg, fe), r
        # eager work on the replayed context between replays
        G.moments(cartesian=True)
    assert torch.isfinite(fg).all()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_wall_loop_with_cleared_inputs_replays_match_eager(precision):
    """The setters' NULL branches (wall shape and wall velocity cleared) are
    kernels too, so a loop that alternates a moving, re-projected wall with a
    wall at rest is capture-safe: every replay matches the eager calls bit for
    bit, with eager work between the replays."""
    lbm = _lbm()
    nx, ny, nz, tau = 40, 12, 6, 0.8
    H = ny - 2
    d = synth.gaussian_bump(nx, nz, A=0.6, x0=20, z0=3, sigma=4)
    v = np.zeros((nz, nx, 3))
    v[..., 0] = 0.01
    side = torch.cuda.Stream()

    def make(stream):
        S = lbm.Solver(nx, ny, nz, tau, precision, stream=stream)
        S.set_body_force((1e-5, 0, 0))
        S.set_wall_displacement(1, d)
        S.init_equilibrium()
        return S

    G, E = make(side), make(torch.cuda.Stream())
    dd = torch.as_tensor(d, device=G.device)
    dv = torch.as_tensor(v, device=G.device)
    fg = torch.zeros((2, 3), dtype=torch.float64, device=G.device)
    fe = torch.zeros((2, 3), dtype=torch.float64, device=G.device)

    def calls(S, force):
        lbm.lbm_set_wall_displacement(S.ctx, 1, None, 1)  # flat wall, re-projected
        lbm.lbm_set_wall_velocity(S.ctx, 1, dv)
        lbm.lbm_step(S.ctx, 2)
        lbm.lbm_wall_force(S.ctx, 1, force[0])
        lbm.lbm_set_wall_displacement(S.ctx, 1, dd, 1)  # bump back, re-projected
        lbm.lbm_set_wall_velocity(S.ctx, 1, None)  # wall at rest
        lbm.lbm_step(S.ctx, 2)
        lbm.lbm_wall_force(S.ctx, 1, force[1])

    calls(G, fg)
    calls(E, fe)
    G.sync()
    E.sync()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        calls(G, fg)
    torch.cuda.synchronize()
    for r in range(3):
        graph.replay()
        torch.cuda.synchronize()
        calls(E, fe)
        E.sync()
        G.sync()
        pg, pe = G.populations(), E.populations()
        assert torch.equal(pg, pe), (r, float((pg - pe).abs().max()))
        assert torch.equal(fg, fe), r
        G.moments(cartesian=True)
    assert torch.isfinite(fg).all()
