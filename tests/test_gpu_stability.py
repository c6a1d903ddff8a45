"""Stability against the depth of a wall concavity (Sec. V.C, stability analysis).

A 128x64x64 channel (H = 62 fluid layers), body force 1e-6 along x, with a
Gaussian concavity (sigma = 8) pushed into the top wall at its centre; the
depth is swept as a fraction of H.  The paper finds its FEM-walled channel
well behaved up to 10 % of the height, with stable spurious effects at 11 %
and an instability by step 140 at 12 %.  Here the run either reaches a steady
state (max pressure deviation settled over 20000 steps) or the instability
guard trips; the maximum pressure at steady state grows with the depth.
"""
import numpy as np
import pytest

from conftest import PAPER
from paper_1803_07822_amd import synth

pytestmark = pytest.mark.gpu

STABLE, UNSTABLE = PAPER["stable_concavity_fraction"], PAPER["unstable_concavity_fraction"]

torch = pytest.importorskip("torch")

NX, NY, NZ = 128, 64, 64
H = NY - 2


def _lbm():
    from paper_1803_07822_amd import lbm

    return lbm


def _run(tau, frac, steps, chunk):
    """(steady max pressure deviation, max |u|) or the step window in which
    the guard tripped."""
    lbm = _lbm()
    d = synth.gaussian_bump(NX, NZ, A=frac * H, x0=NX / 2, z0=NZ / 2, sigma=8.0)
    S = lbm.Solver(NX, NY, NZ, tau, "fp32")
    S.set_body_force((1e-6, 0.0, 0.0))
    S.set_wall_displacement(1, d)
    S.init_equilibrium()
    done, out = 0, None
    while done < steps:
        try:
            S.step(chunk)
            S.sync()
        except lbm.LBMError as e:
            assert e.code == -5
            out = ("tripped", done, done + chunk)
            break
        done += chunk
    if out is None:
        r, u = S.moments(cartesian=True)
        out = ("steady", float((r - 1).abs().max()) / 3.0, float(u.abs().max()))
    del S
    torch.cuda.empty_cache()
    return out


@pytest.mark.parametrize("tau,stable,unstable", [(1.0, [0.02, 0.04, 0.06, 0.08, 0.09, STABLE, 0.11], [UNSTABLE]),
                                                 (0.8, [0.04, 0.08, 0.09], [0.10]),
                                                 (0.6, [0.02, 0.04], [0.06])])
def test_concavity_depth_sweep(tau, stable, unstable):
    res = {}
    for f in stable:
        res[f] = _run(tau, f, 20000, 1000)
    for f in unstable:
        res[f] = _run(tau, f, 2000, 10)
    print(f"tau {tau}:", {f"{k:.2f}": (v[0], f"{v[1]:.3g}", f"{v[2]:.3g}") for k, v in res.items()}, flush=True)
    for f in stable:
        assert res[f][0] == "steady", (f, res[f])
    for f in unstable:
        assert res[f][0] == "tripped", (f, res[f])
    dp = [res[f][1] for f in stable]
    assert all(np.diff(dp) > 0), dp  # deeper concavity, higher peak pressure
    if tau == 1.0:
        # the paper's thresholds: stable at its bound, unstable at its
        # instability depth, and within twice the step it shows that at
        assert res[UNSTABLE][2] <= 2 * PAPER["unstable_by_step"], res[UNSTABLE]
