"""lbm_wall_force_noalloc (the wall force with its reduction scratch in the
library's static device array) against lbm_wall_force (scratch in the
context's workspace), through the C-ABI: two calls in a row, the second on a
smaller grid, and the size limit."""
import numpy as np
import pytest

from paper_1803_07822_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lbm():
    from paper_1803_07822_amd import lbm

    return lbm


def _solver(nx, ny, nz, precision, seed):
    lbm = _lbm()
    S = lbm.Solver(nx, ny, nz, 0.7, precision)
    S.set_body_force((1e-5, 0.0, 2e-6))
    S.set_wall_displacement(1, synth.gaussian_bump(nx, nz, A=0.3 * (ny - 2) / 8, x0=nx / 2, z0=nz / 3, sigma=3))
    S.init_equilibrium(None, synth.uniform_noise_velocity(nx, ny, nz, 1e-3, seed=seed))
    S.step(4)
    return S


def _both(S, wall, method):
    lbm = _lbm()
    out = []
    for fn in (lbm.lbm_wall_force, lbm.lbm_wall_force_noalloc):
        tot = torch.full((3,), float("nan"), dtype=torch.float64, device=S.device)
        pn = torch.full((S.nz, S.nx, 3), float("nan"), dtype=torch.float64, device=S.device)
        fn(S.ctx, wall, tot, pn, method)
        S.sync()
        out.append((tot.cpu().numpy(), pn.cpu().numpy()))
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_wall_force_matches_workspace_wall_force(precision):
    lbm = _lbm()
    for nx, ny, nz, seed in ((150, 10, 44, 2), (40, 8, 12, 3)):  # 6600 then 480 wall columns
        S = _solver(nx, ny, nz, precision, seed)
        for wall, method in ((1, lbm.LBM_FORCE_STRESS), (0, lbm.LBM_FORCE_STRESS), (1, lbm.LBM_FORCE_MEM)):
            (t0, p0), (t1, p1) = _both(S, wall, method)
            assert np.isfinite(t0).all() and np.isfinite(p0).all()
            assert np.abs(t0).max() > 0
            # same kernel, same reduction order: identical to the last bit
            assert np.array_equal(t0, t1), (nx, wall, method, t0, t1)
            assert np.array_equal(p0, p1)
        del S


def test_noalloc_wall_force_size_limit():
    lbm = _lbm()
    nx, nz = 2048, lbm.LBM_NOALLOC_MAX_COLUMNS // 2048 + 1  # one column row too many
    S = lbm.Solver(nx, 4, nz, 0.8, "fp32")
    tot = torch.empty(3, dtype=torch.float64, device=S.device)
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_wall_force_noalloc(S.ctx, 1, tot)
    assert e.value.code == -1  # LBM_EINVAL
