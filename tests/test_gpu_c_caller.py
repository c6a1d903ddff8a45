"""The C-ABI from a plain C++ caller (tests/c_caller/lbm_c_caller.cpp: only
include/lbm.h and the HIP runtime, no Python or torch), against the same
calls made through the Python binding: identical results, bit for bit, and
the call order enforced (a step before any state is refused)."""
import json
import os
import subprocess

import numpy as np
import pytest

from paper_1803_07822_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CALLER = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_caller", "lbm_c_caller")


def test_plain_caller_matches_python_binding(tmp_path):
    from paper_1803_07822_amd import lbm

    if not os.path.exists(CALLER):
        pytest.fail(f"{CALLER} is missing: build it with __graft_entry__.build()")
    w = synth.workload("c1_shear_32x16x16")
    nx, ny, nz, H, steps = w.nx, w.ny, w.nz, w.ny - 2, 300
    d = np.ascontiguousarray(w.disp(), dtype=np.float64)
    d.tofile(tmp_path / "disp.bin")
    r = subprocess.run([CALLER, str(tmp_path / "disp.bin"), str(steps), str(tmp_path / "out.bin")],
                       capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stderr
    info = json.loads([ln for ln in r.stdout.splitlines() if ln.startswith("{")][-1])
    assert info["status"] == 0 and info["early_step"] == -4  # LBM_OK; the early step: LBM_ESTATE
    nf = nx * H * nz
    out = np.fromfile(tmp_path / "out.bin", dtype=np.float64)
    assert out.size == 4 * nf + 3 + 12
    rho_c = out[:nf].reshape(nz, H, nx)
    u_c = out[nf:4 * nf].reshape(3, nz, H, nx)
    f_c = out[4 * nf:4 * nf + 3]
    fs_c = out[4 * nf + 3:].reshape(4, 3)

    S = lbm.Solver(nx, ny, nz, w.tau, "fp64")
    S.set_body_force(w.force)
    S.set_wall_displacement(lbm.LBM_WALL_YMAX, d)
    S.init_equilibrium()
    S.step(steps)
    rho, u = S.moments(cartesian=True)
    force = S.wall_force(lbm.LBM_WALL_YMAX)
    assert np.array_equal(rho_c, rho.cpu().numpy())
    assert np.array_equal(u_c, u.cpu().numpy())
    assert np.array_equal(f_c, force.cpu().numpy())
    assert np.abs(u_c).max() > 0  # the drive has set up a flow
    # four more steps, each with the top-wall force of the state it starts from
    fs = torch.empty((4, 3), dtype=torch.float64, device=S.device)
    lbm.lbm_step_force(S.ctx, 4, lbm.LBM_WALL_YMAX, fs)
    S.sync()
    assert np.array_equal(fs_c, fs.cpu().numpy())
    # the first of them is the state the force above was taken from
    assert np.abs(fs_c[0] - f_c).max() <= 1e-13 * np.abs(f_c).max()
