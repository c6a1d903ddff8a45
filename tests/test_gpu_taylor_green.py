"""Taylor-Green vortex under a time-dependent diagonal metric (Sec. V.A).

The vortex lives in the periodic (x, z) plane of the channel:
u_c = v0 exp(-2 nu k^2 t) (sin k x_c cos k z_c, 0, -cos k x_c sin k z_c),
k = 2 pi / L, the closed-form decay of the incompressible Navier-Stokes
equations.  The chart x_c = xi_x + eps sin(2 pi xi_x / L - eta t) (and the same
in z) moves every step and the state is re-projected every step, as the paper
does.  The channel is 2L high so that the no-slip walls in y stay out of
reach of the mid-plane over one half-life of the vortex (the wall's influence
there is erfc(5.3) ~ 1e-13 of the amplitude).

Scaling with resolution L (diffusive): tau = 0.8 fixed, v0 = 20 nu / L
(Re = 20), eps = 0.1 L/32, eta = 0.05 (32/L)^2, run to one half-life
t = ln 2 / (2 nu k^2).
"""
import math

import numpy as np
import pytest

from oracle import Oracle
from paper_1803_07822_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
TAU = 0.8
NU = (TAU - 0.5) / 3.0


def _lbm():
    from paper_1803_07822_amd import lbm

    return lbm


def _tg_rho(chart, v0):
    """Density of the Taylor-Green pressure field, rho = 1 + p / c_s^2 with
    p = -(v0^2 / 4)(cos 2 k x_c + cos 2 k z_c)."""
    nx, nz = chart.shape[3], chart.shape[1]
    xc, zc = chart[0][:, 1:-1, :], chart[2][:, 1:-1, :]
    return 1.0 - 0.75 * v0**2 * (np.cos(4 * np.pi * xc / nx) + np.cos(4 * np.pi * zc / nz))


def _params(L, moving=True):
    v0 = 20.0 * NU / L
    eps = 0.1 * L / 32.0 if moving else 0.0
    eta = 0.05 * (32.0 / L) ** 2
    k = 2 * math.pi / L
    steps = int(round(math.log(2.0) / (2 * NU * k * k)))
    return v0, eps, eta, k, steps


def _chart_dev(L, ny, eps, eta, t, device):
    """synth.taylor_green_chart built on the device (one per step would
    otherwise cost more host time than the run)."""
    i = torch.arange(L, dtype=torch.float64, device=device)
    ch = torch.empty((3, L, ny, L), dtype=torch.float64, device=device)
    ch[0] = (i + eps * torch.sin(2 * math.pi * i / L - eta * t))[None, None, :]
    ch[1] = torch.arange(ny, dtype=torch.float64, device=device)[None, :, None]
    ch[2] = (i + eps * torch.sin(2 * math.pi * i / L - eta * t))[:, None, None]
    return ch


def _run(S, L, moving=True):
    nx = nz = L
    ny = 2 * L + 2
    v0, eps, eta, k, steps = _params(L, moving)
    ch = synth.taylor_green_chart(nx, ny, nz, eps, eta, 0.0)
    assert np.abs(_chart_dev(L, ny, eps, eta, 0.0, S.device).cpu().numpy() - ch).max() < 1e-12
    S.set_body_force((0.0, 0.0, 0.0))
    S.set_metric(ch)
    S.init_equilibrium(_tg_rho(ch, v0), synth.taylor_green_velocity(ch, v0))
    for t in range(1, steps + 1):
        S.step(1)
        if moving:
            S.set_metric(_chart_dev(L, ny, eps, eta, float(t), S.device), reproject=True)
    return steps


def _error(S, L, steps, moving=True):
    """Relative L2 error of the Cartesian velocity on the mid-plane layer
    against the decayed closed form at the node positions, and the relative
    error of the vortex amplitude (the field's projection on the closed
    form)."""
    nx = nz = L
    ny = 2 * L + 2
    v0, eps, eta, k, _ = _params(L, moving)
    ch = synth.taylor_green_chart(nx, ny, nz, eps, eta, float(steps))
    _, u = S.moments(cartesian=True)
    u = u.cpu().numpy()
    jm = L  # fluid layer at the channel's middle
    xc, zc = ch[0][:, jm + 1, :], ch[2][:, jm + 1, :]
    a = v0 * math.exp(-2 * NU * k * k * steps)
    ux, uz = a * np.sin(k * xc) * np.cos(k * zc), -a * np.cos(k * xc) * np.sin(k * zc)
    num = np.sqrt(((u[0][:, jm, :] - ux) ** 2 + (u[2][:, jm, :] - uz) ** 2 + u[1][:, jm, :] ** 2).sum())
    den = np.sqrt((ux**2 + uz**2).sum())
    amp = ((u[0][:, jm, :] * ux).sum() + (u[2][:, jm, :] * uz).sum()) / (den * den)
    return num / den, abs(amp - 1.0)


def test_taylor_green_moving_chart_parity_fp64():
    """Small Taylor-Green case with the chart moved and the state re-projected
    every step: GPU FP64 against the oracle, population by population."""
    lbm = _lbm()
    L, steps = 16, 6
    nx = nz = L
    ny = 2 * L + 2
    v0, eps, eta, _, _ = _params(L)
    ch = synth.taylor_green_chart(nx, ny, nz, eps, eta, 0.0)
    S = lbm.Solver(nx, ny, nz, TAU, "fp64")
    O = Oracle(nx, ny, nz, TAU)
    for X in (S, O):
        X.set_body_force((0.0, 0.0, 0.0))
        X.set_metric(ch)
        X.init_equilibrium(_tg_rho(ch, v0), synth.taylor_green_velocity(ch, v0))
    for t in range(1, steps + 1):
        cht = synth.taylor_green_chart(nx, ny, nz, eps, eta, float(t))
        for X in (S, O):
            X.step(1)
            X.set_metric(cht, reproject=True)
    fo = O.populations()
    err = np.abs(S.populations().cpu().numpy() - fo).max() / np.abs(fo - W[:, None, None, None]).max()
    assert err < 1e-12, err


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_taylor_green_decay_converges(precision):
    """Error against the closed-form decay after one half-life, L = 32, 64,
    128, with the chart moving every step.  It falls with resolution at
    first order: the trilinear re-projection error accumulates as half the
    chart's total travel times |u''|, which is O(1/L) in this scaling.  The
    same runs on the fixed identity chart fall at second order."""
    lbm = _lbm()
    errs, amps, flat = {}, {}, {}
    for L in (32, 64, 128):
        for moving in (True, False):
            S = lbm.Solver(L, 2 * L + 2, L, TAU, precision)
            steps = _run(S, L, moving)
            e, a = _error(S, L, steps, moving)
            if moving:
                errs[L], amps[L] = e, a
            else:
                flat[L] = (e, a)
            del S
            torch.cuda.empty_cache()
    print(f"Taylor-Green {precision}: moving chart L2", {k: f"{v:.3e}" for k, v in errs.items()},
          "amplitude", {k: f"{v:.3e}" for k, v in amps.items()},
          "| fixed flat chart (L2, amplitude)", {k: f"{v[0]:.3e}, {v[1]:.3e}" for k, v in flat.items()}, flush=True)
    assert errs[32] / errs[64] > 1.7 and errs[64] / errs[128] > 1.7, errs
    assert errs[128] < 5e-3, errs
    assert amps[32] / amps[64] > 1.7 and amps[64] / amps[128] > 1.7, amps
    assert amps[128] < 5e-3, amps
    # on the fixed chart the scheme's own error falls at second order
    assert flat[64][1] / flat[128][1] > 3.0, flat
