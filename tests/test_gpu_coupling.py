"""Coupling interface (lbm_couple): a closed fluid-structure loop with a toy
structure, run through the GPU library and, call by call, through the oracle.

The structure is one damped oscillator per wall column for the top wall's
normal displacement d: d'' = -w^2 d - c d' + k (f_y - p0), driven by the
fluid's normal force per column f_y above the reference p0 = 1/3 (rho theta
at rho = 1).  Each coupling interval hands the structure's new displacement
and velocity to the fluid (with re-projection), advances n LBM steps and
returns the traction; the oscillator then advances one interval with a
semi-implicit Euler step.  (With a lighter structure, k = 1, the loop shows
the added-mass instability of partitioned coupling within 5 intervals; the
parameters here keep it stable while the wall relaxes visibly.)
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


def _structure_step(d, v, fy, dt, w2=2e-3, c=0.05, k=0.2, p0=1.0 / 3.0):
    a = -w2 * d - c * v + k * (fy - p0)
    v = v + dt * a
    return d + dt * v, v


def _velocity(v):
    out = np.zeros(v.shape + (3,))
    out[..., 1] = v
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_coupled_loop_matches_oracle(precision):
    lbm = _lbm()
    nx, ny, nz, tau, n, intervals = 24, 10, 16, 0.8, 4, 6
    d = synth.gaussian_bump(nx, nz, A=0.3, x0=12.0, z0=8.0, sigma=4.0)
    v = np.zeros_like(d)
    S = lbm.Solver(nx, ny, nz, tau, precision)
    O = Oracle(nx, ny, nz, tau)
    for X in (S, O):
        X.set_body_force((1e-5, 0.0, 0.0))
        X.set_wall_displacement(1, d)
        X.init_equilibrium()
    dg, vg = d.copy(), v.copy()
    for it in range(intervals):
        tot, pn = S.couple(1, dg if it else None, _velocity(vg), n)
        pn = pn.cpu().numpy()
        if it:
            O.set_wall_displacement(1, d, reproject=True)
        O.set_wall_velocity(1, _velocity(v))
        O.step(n)
        to, pno = O.wall_force(1, per_node=True)
        if precision == "fp64":
            assert np.abs(pn - pno).max() < 1e-12 * np.abs(pno).max(), it
            assert np.abs(tot.cpu().numpy() - to).max() < 1e-12 * np.abs(to).max(), it
        else:
            assert np.abs(pn - pno).max() < 1e-5 * np.abs(pno).max(), it
        dg, vg = _structure_step(dg, vg, pn[..., 1], float(n))
        d, v = _structure_step(d, v, pno[..., 1], float(n))
    print(precision, "coupled loop: max |d_gpu - d_oracle|", np.abs(dg - d).max(), "max |d|", np.abs(d).max(),
          "max |v|", np.abs(v).max(), flush=True)
    assert np.abs(v).max() > 1e-4  # the wall actually moved under the fluid load
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert np.abs(dg - d).max() < tol * np.abs(d).max()
    fo = O.populations()
    if precision == "fp64":
        assert np.abs(S.populations().cpu().numpy() - fo).max() < 1e-12 * np.abs(fo - W[:, None, None, None]).max()


def test_couple_argument_errors():
    lbm = _lbm()
    S = lbm.Solver(8, 6, 4, 0.8)
    tot = torch.zeros(3, dtype=torch.float64, device=S.device)
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_couple(S.ctx, 1, None, None, 1, tot)
    assert e.value.code == -4  # no state yet
    S.set_wall_displacement(1, np.zeros((4, 8)))
    S.init_equilibrium()
    for wall, n, t in ((2, 1, tot), (1, -1, tot), (1, 1, None)):
        with pytest.raises(lbm.LBMError) as e:
            lbm.lbm_couple(S.ctx, wall, None, None, n, t)
        assert e.value.code == -1
