"""Pins of the oracle's open ends in x (Sec. VI.A: inlet and outlet by
extrapolation from the inner neighbours, the inlet with a prescribed
velocity profile).  The streamed part of the incoming populations is
extrapolated linearly from the two next columns in: a copy (zero gradient)
from one column admits no steady pressure gradient through the outlet, and
the channel then fills up (its density grows without bound under a
velocity inlet), while the linear form passes the linear pressure drop of
a developed channel flow.

Each test checks the oracle against something fixed from outside it: an
exact steady state that the extrapolation must leave alone, the textbook
flat D3Q19 equilibrium written here independently, and the pressure drop of
pressure-driven Poiseuille flow.
"""
import numpy as np
import pytest

from oracle import Oracle

CS2 = 1.0 / 3.0
C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
              [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def steady_steps(H, tau, n_decay=25.0):
    nu = (tau - 0.5) / 3
    return int(n_decay / (nu * (np.pi / H) ** 2))


def textbook_feq(rho, u):
    """Flat D3Q19 equilibrium, rho w (1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2))."""
    cu = np.tensordot(C, u, axes=(1, 0))
    uu = (u * u).sum(axis=0)
    return W.reshape((19,) + (1,) * rho.ndim) * rho * (1 + cu / CS2 + cu**2 / (2 * CS2**2) - uu / (2 * CS2))


def test_open_ends_leave_a_developed_channel_flow_unchanged():
    """The exact steady state of the periodic body-force channel is invariant
    along x; opening the ends with that profile as the inlet velocity (and
    the same body force) leaves it unchanged: the outlet copy and the inlet
    extrapolation are exact on an x-invariant state, and the inlet
    correction vanishes when the prescribed velocity is the inner one."""
    nx, H, nz, tau, F = 6, 8, 2, 0.8, 1e-5
    o = Oracle(nx, H + 2, nz, tau)
    o.set_body_force([F, 0, 0])
    o.set_wall_displacement(1, np.zeros((nz, nx)))
    o.init_equilibrium()
    o.step(steady_steps(H, tau, 40))
    f = o.populations()
    _, u = o.moments(cartesian=True)
    uin = np.moveaxis(u[:, :, :, 0], 0, -1)  # [nz, H, 3] from column 0
    q = Oracle(nx, H + 2, nz, tau)
    q.set_body_force([F, 0, 0])
    q.set_open_x(uin)
    q.set_wall_displacement(1, np.zeros((nz, nx)))
    q.set_populations(f)
    assert np.abs(q.populations() - f).max() < 1e-15
    q.step(100)
    assert np.abs(q.populations() - f).max() < 1e-13


def test_inlet_populations_are_the_equilibrium_of_the_prescribed_velocity():
    """A uniform flat equilibrium state (rho1, u1) with a different inlet
    velocity u_in: the populations entering at the inlet become the textbook
    equilibrium f^eq(rho1, u_in) (density extrapolated, velocity imposed,
    zero non-equilibrium part), the others stay; the outlet keeps
    f^eq(rho1, u1)."""
    nx, H, nz = 6, 4, 3
    r1, u1 = 1.02, np.array([0.03, -0.004, 0.01])
    uin = np.array([0.05, 0.002, -0.007])
    o = Oracle(nx, H + 2, nz, 0.7)
    o.set_open_x(np.broadcast_to(uin, (nz, H, 3)).copy())
    o.set_wall_displacement(1, np.zeros((nz, nx)))
    rho = np.full((nz, H, nx), r1)
    ucart = np.broadcast_to(u1[:, None, None, None], (3, nz, H, nx)).copy()
    o.init_equilibrium(rho, ucart)
    f = o.populations()
    feq1 = textbook_feq(np.array(r1), u1)
    feqin = textbook_feq(np.array(r1), uin)
    inc = C[:, 0] > 0
    assert np.abs(f[inc][:, :, :, 0] - feqin[inc][:, None, None]).max() < 1e-15
    assert np.abs(f[~inc][:, :, :, 0] - feq1[~inc][:, None, None]).max() < 1e-15
    assert np.abs(f[:, :, :, 1:] - feq1[:, None, None, None]).max() < 1e-15


def test_pressure_driven_poiseuille_between_open_ends():
    """No body force: the inlet imposes the developed parabola of peak U and
    the outlet is open.  At steady state the mass flux is the same through
    every column, the profile stays that parabola along the channel, and the
    pressure falls linearly with the slope G of plane Poiseuille flow
    carrying the same flux.  For BGK with halfway bounce-back the profile of
    a gradient G is G/(2 rho nu) [eta (H - eta) + (16 L - 3)/12]
    (L = (tau - 1/2)^2, the wall pin's closed form), so matching the flux of
    the parabola gives G = 8 rho nu U / H^2 * S / (S + H (16 L - 3)/12) with
    S = sum eta (H - eta) (to the O(Ma^2) compressibility of the lattice
    fluid)."""
    nx, H, nz, tau, U = 40, 10, 1, 0.8, 2e-3
    nu = (tau - 0.5) / 3
    eta = np.arange(H) + 0.5
    prof = 4 * U * eta * (H - eta) / H**2
    uin = np.zeros((nz, H, 3))
    uin[..., 0] = prof[None, :]
    o = Oracle(nx, H + 2, nz, tau)
    o.set_open_x(uin)
    o.set_wall_displacement(1, np.zeros((nz, nx)))
    ucart = np.zeros((3, nz, H, nx))
    ucart[0] = prof[None, :, None]
    o.init_equilibrium(None, ucart)
    o.step(steady_steps(max(H, nx // 2), tau, 12))
    rho, u = o.moments(cartesian=True)
    flux = (rho[0] * u[0][0]).sum(axis=0)
    assert np.abs(flux / flux[0] - 1).max() < 1e-8  # steady: the same mass flux through every column
    o.step(500)
    assert np.abs(o.moments()[0] - rho).max() < 1e-8  # and the density level holds
    mid = slice(10, 30)
    assert np.abs(u[0][0, :, mid] - prof[:, None]).max() < 1e-2 * U
    p = rho[0].mean(axis=0) / 3.0
    slope = np.polyfit(np.arange(nx)[mid], p[mid], 1)[0]
    S = (eta * (H - eta)).sum()
    lam = (tau - 0.5) ** 2
    expect = -rho[0][:, mid].mean() * 8 * nu * U / H**2 * S / (S + H * (16 * lam - 3) / 12)
    print("pressure slope", slope, "expected", expect)
    assert abs(slope / expect - 1) < 2e-3, (slope, expect)
