"""ctypes binding of ``liblbm.so`` (C-ABI in ``include/lbm.h``).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch supplies device memory (the workspace and all arrays) and the stream.
Importing this module fails if the library has not been built.

Low-level functions carry the C names (``lbm_create``, ``lbm_set_metric``,
``lbm_step``, ...) and take a context handle plus torch tensors; ``Solver``
wraps one context with its workspace.
"""
import ctypes
import functools
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first (python -c 'import __graft_entry__ as g; g.build()')"
    )

_lib = ctypes.CDLL(LIB_PATH)

LBM_D3Q19 = 19
LBM_FP64, LBM_FP32_DEV = 0, 1
LBM_WALL_YMIN, LBM_WALL_YMAX = 0, 1
LBM_FORCE_STRESS = 0
LBM_FORCE_MEM = 1
LBM_NOALLOC_MAX_COLUMNS = 256 * 2048  # lbm_wall_force_noalloc's limit on nx * nz
ERRORS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EHIP", -4: "LBM_ESTATE",
          -5: "LBM_EUNSTABLE", -6: "LBM_EUNSUPPORTED"}

SYMBOLS = [
    "lbm_workspace_bytes", "lbm_create", "lbm_reserve_adjoint", "lbm_destroy", "lbm_set_body_force",
    "lbm_set_metric", "lbm_set_wall_displacement", "lbm_set_wall_velocity", "lbm_init_equilibrium",
    "lbm_set_populations", "lbm_get_populations", "lbm_get_history", "lbm_get_geometry", "lbm_step", "lbm_step_force",
    "lbm_step_profiled", "lbm_set_tuning", "lbm_get_tuning", "lbm_stream_probe", "lbm_moments", "lbm_wall_force",
    "lbm_wall_force_noalloc", "lbm_couple", "lbm_set_plate", "lbm_set_plate_displacement", "lbm_set_plate_velocity", "lbm_plate_force",
    "lbm_set_open_x", "lbm_forward_record", "lbm_backward", "lbm_sync", "lbm_last_error",
]


class lbm_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_lib.lbm_workspace_bytes.restype = ctypes.c_size_t
_lib.lbm_workspace_bytes.argtypes = [ctypes.POINTER(lbm_grid), _I, _I, _I, _I]
_lib.lbm_create.argtypes = [ctypes.POINTER(_P), ctypes.POINTER(lbm_grid), _I, ctypes.c_double, _I, _P,
                            ctypes.c_size_t, _P]
_lib.lbm_reserve_adjoint.argtypes = [_P, _I, _I]
_lib.lbm_destroy.argtypes = [_P]
_lib.lbm_set_body_force.argtypes = [_P, ctypes.POINTER(ctypes.c_double)]
_lib.lbm_set_metric.argtypes = [_P, _P, _I]
_lib.lbm_set_wall_displacement.argtypes = [_P, _I, _P, _I]
_lib.lbm_set_wall_velocity.argtypes = [_P, _I, _P]
_lib.lbm_init_equilibrium.argtypes = [_P, _P, _P]
_lib.lbm_set_populations.argtypes = [_P, _P]
_lib.lbm_get_populations.argtypes = [_P, _P]
_lib.lbm_get_history.argtypes = [_P, _P]
_lib.lbm_get_geometry.argtypes = [_P, _P, _P]
_lib.lbm_step.argtypes = [_P, _I]
_lib.lbm_step_force.argtypes = [_P, _I, _I, _P]
_lib.lbm_step_profiled.argtypes = [_P, _I, ctypes.POINTER(ctypes.c_double), _I]
_lib.lbm_set_tuning.argtypes = [_P, _I, _I, _I]
_lib.lbm_stream_probe.argtypes = [_I, ctypes.c_longlong, _P, _P, _P]
_lib.lbm_get_tuning.argtypes = [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int)]
_lib.lbm_moments.argtypes = [_P, _P, _P, _I]
_lib.lbm_wall_force.argtypes = [_P, _I, _I, _P, _P]
_lib.lbm_wall_force_noalloc.argtypes = [_P, _I, _I, _P, _P]
_lib.lbm_set_plate.argtypes = [_P, _I, _I, _I]
_lib.lbm_set_plate_displacement.argtypes = [_P, _P, _I]
_lib.lbm_set_plate_velocity.argtypes = [_P, _P]
_lib.lbm_plate_force.argtypes = [_P, _P, _P]
_lib.lbm_set_open_x.argtypes = [_P, _P]
_lib.lbm_forward_record.argtypes = [_P, _I, _I, _I, _I, _P]
_lib.lbm_backward.argtypes = [_P, _P, _P, _P, _P]
_lib.lbm_sync.argtypes = [_P]
_lib.lbm_last_error.restype = ctypes.c_char_p
_lib.lbm_last_error.argtypes = [_P]
for _n in SYMBOLS:
    if _n not in ("lbm_workspace_bytes", "lbm_last_error"):
        getattr(_lib, _n).restype = _I


class LBMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("device arrays must be torch tensors")
    if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("device arrays must be contiguous float64 tensors on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _check(ctx, code):
    if code != 0:
        raise LBMError(code, lbm_last_error(ctx))
    return code


# ------------------------------------------------------- C names, thin wrappers
def lbm_workspace_bytes(nx, ny, nz, precision=LBM_FP64, adjoint_K=0, ckpt_every=0, lattice=LBM_D3Q19):
    g = lbm_grid(nx, ny, nz)
    return int(_lib.lbm_workspace_bytes(ctypes.byref(g), lattice, precision, adjoint_K, ckpt_every))


def lbm_create(nx, ny, nz, tau, precision, workspace: torch.Tensor, stream=None, lattice=LBM_D3Q19):
    g = lbm_grid(nx, ny, nz)
    h = _P()
    st = ctypes.c_void_p(stream if stream is not None else torch.cuda.current_stream().cuda_stream)
    code = _lib.lbm_create(ctypes.byref(h), ctypes.byref(g), lattice, float(tau), precision,
                           ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(), st)
    if code != 0:
        raise LBMError(code, "lbm_create failed")
    return h


def lbm_last_error(ctx):
    m = _lib.lbm_last_error(ctx)
    return m.decode() if m else ""


def lbm_reserve_adjoint(ctx, K, ckpt_every):
    return _check(ctx, _lib.lbm_reserve_adjoint(ctx, int(K), int(ckpt_every)))


def lbm_destroy(ctx):
    return _lib.lbm_destroy(ctx)


def lbm_set_body_force(ctx, F):
    arr = (ctypes.c_double * 3)(*[float(v) for v in F])
    return _check(ctx, _lib.lbm_set_body_force(ctx, arr))


def lbm_set_metric(ctx, chart, reproject=False):
    return _check(ctx, _lib.lbm_set_metric(ctx, _ptr(chart), int(bool(reproject))))


def lbm_set_wall_displacement(ctx, wall, d, reproject=False):
    return _check(ctx, _lib.lbm_set_wall_displacement(ctx, int(wall), _ptr(d), int(bool(reproject))))


def lbm_set_wall_velocity(ctx, wall, v):
    return _check(ctx, _lib.lbm_set_wall_velocity(ctx, int(wall), _ptr(v)))


def lbm_set_plate(ctx, jp, i0, i1):
    return _check(ctx, _lib.lbm_set_plate(ctx, int(jp), int(i0), int(i1)))


def lbm_set_plate_displacement(ctx, d, reproject=False):
    return _check(ctx, _lib.lbm_set_plate_displacement(ctx, _ptr(d), int(bool(reproject))))


def lbm_set_plate_velocity(ctx, v):
    return _check(ctx, _lib.lbm_set_plate_velocity(ctx, _ptr(v)))


def lbm_plate_force(ctx, total, per_column=None):
    return _check(ctx, _lib.lbm_plate_force(ctx, _ptr(total), _ptr(per_column)))


def lbm_set_open_x(ctx, uin):
    return _check(ctx, _lib.lbm_set_open_x(ctx, _ptr(uin)))


def lbm_init_equilibrium(ctx, rho=None, ucart=None):
    return _check(ctx, _lib.lbm_init_equilibrium(ctx, _ptr(rho), _ptr(ucart)))


def lbm_set_populations(ctx, f):
    return _check(ctx, _lib.lbm_set_populations(ctx, _ptr(f)))


def lbm_get_populations(ctx, out):
    return _check(ctx, _lib.lbm_get_populations(ctx, _ptr(out)))


def lbm_get_history(ctx, out):
    return _check(ctx, _lib.lbm_get_history(ctx, _ptr(out)))


def lbm_get_geometry(ctx, geo, jac=None):
    return _check(ctx, _lib.lbm_get_geometry(ctx, _ptr(geo), _ptr(jac)))


def lbm_step(ctx, n=1):
    return _check(ctx, _lib.lbm_step(ctx, int(n)))


def lbm_step_force(ctx, n, wall, forces):
    """n steps; forces [n, 3] (device, FP64) receives the force on `wall` of
    each state stepped from."""
    return _check(ctx, _lib.lbm_step_force(ctx, int(n), int(wall), _ptr(forces)))


def lbm_step_profiled(ctx, n, nslots=4):
    """Run n steps; returns the average duration (ms) of each kernel of the step."""
    arr = (ctypes.c_double * nslots)()
    _check(ctx, _lib.lbm_step_profiled(ctx, int(n), arr, nslots))
    return list(arr)


def lbm_set_tuning(ctx, zchunk=0, variant=0, stage=-1):
    return _check(ctx, _lib.lbm_set_tuning(ctx, int(zchunk), int(variant), int(stage)))


def lbm_stream_probe(precision, n, d_in, d_out, stream):
    """Bandwidth calibration kernel (see include/lbm.h); no context.  d_in
    ([57 n]) and d_out ([29 n]) are contiguous GPU tensors of float64 for
    LBM_FP64, float32 for LBM_FP32_DEV."""
    dt = torch.float64 if precision == LBM_FP64 else torch.float32
    for t, m in ((d_in, 57), (d_out, 29)):
        if not (t.is_cuda and t.is_contiguous() and t.dtype == dt and t.numel() >= m * n):
            raise ValueError("probe buffers must be contiguous GPU tensors of the precision's type and size")
    rc = _lib.lbm_stream_probe(int(precision), int(n), ctypes.c_void_p(d_in.data_ptr()),
                               ctypes.c_void_p(d_out.data_ptr()), ctypes.c_void_p(stream))
    if rc != 0:
        raise LBMError(rc, "lbm_stream_probe")
    return rc


def lbm_get_tuning(ctx):
    """(zchunk, variant, stage) the next step runs with."""
    z, v, st = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
    _check(ctx, _lib.lbm_get_tuning(ctx, ctypes.byref(z), ctypes.byref(v), ctypes.byref(st)))
    return z.value, v.value, st.value


def lbm_moments(ctx, rho, u, cartesian=False):
    return _check(ctx, _lib.lbm_moments(ctx, _ptr(rho), _ptr(u), int(bool(cartesian))))


def lbm_wall_force(ctx, wall, total, per_node=None, method=LBM_FORCE_STRESS):
    return _check(ctx, _lib.lbm_wall_force(ctx, int(wall), int(method), _ptr(total), _ptr(per_node)))


def lbm_wall_force_noalloc(ctx, wall, total, per_node=None, method=LBM_FORCE_STRESS):
    return _check(ctx, _lib.lbm_wall_force_noalloc(ctx, int(wall), int(method), _ptr(total), _ptr(per_node)))


def lbm_couple(ctx, wall, disp, vcart, n, total, per_node=None):
    return _check(ctx, _lib.lbm_couple(ctx, int(wall), _ptr(disp), _ptr(vcart), int(n), _ptr(total),
                                       _ptr(per_node)))


def lbm_forward_record(ctx, K, ckpt_every, wall, forces, method=LBM_FORCE_STRESS):
    return _check(ctx, _lib.lbm_forward_record(ctx, int(K), int(ckpt_every), int(wall), int(method), _ptr(forces)))


def lbm_backward(ctx, dLdF, grad_disp=None, grad_chart=None, grad_f0=None):
    return _check(ctx, _lib.lbm_backward(ctx, _ptr(dLdF), _ptr(grad_disp), _ptr(grad_chart), _ptr(grad_f0)))


def lbm_sync(ctx):
    return _check(ctx, _lib.lbm_sync(ctx))


# ------------------------------------------------------------------ Solver
class Solver:
    """One context with its workspace on ``device`` (a CUDA/HIP torch device)."""

    def __init__(self, nx, ny, nz, tau, precision="fp64", adjoint_K=0, ckpt_every=0, device="cuda:0", stream=None):
        """stream: the torch stream the context enqueues on (default: the
        device's current stream).  A stream of its own lets a caller capture
        a sequence of calls into a HIP graph and replay it."""
        self.nx, self.ny, self.nz, self.tau = nx, ny, nz, tau
        self.H = ny - 2
        self.device = torch.device(device)
        self.precision = {"fp64": LBM_FP64, "fp32": LBM_FP32_DEV}[precision]
        nbytes = lbm_workspace_bytes(nx, ny, nz, self.precision, adjoint_K, ckpt_every)
        if nbytes == 0:
            raise ValueError("invalid grid or adjoint sizes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.ctx = lbm_create(nx, ny, nz, tau, self.precision, self.workspace, self.stream.cuda_stream)
        if adjoint_K:
            lbm_reserve_adjoint(self.ctx, adjoint_K, ckpt_every)
        self.adjoint_K, self.ckpt_every = adjoint_K, ckpt_every
        self.recordings = 0  # forward_record calls so far

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx and _lib is not None:
            try:
                _lib.lbm_destroy(ctx)
            except Exception:  # interpreter shutdown: the library may be gone
                pass
            self.ctx = None

    @property
    def fluid_shape(self):
        return (self.nz, self.H, self.nx)

    @property
    def fluid_nodes(self):
        return self.nz * self.H * self.nx

    def _dev(self, a, shape=None):
        if a is None:
            return None
        t = torch.as_tensor(a, dtype=torch.float64).to(self.device).contiguous()
        if shape is not None:
            t = t.reshape(shape)
        return t

    def set_body_force(self, F):
        lbm_set_body_force(self.ctx, F)

    def set_metric(self, chart, reproject=False):
        self._keep = self._dev(chart, (3, self.nz, self.ny, self.nx))
        lbm_set_metric(self.ctx, self._keep, reproject)

    def set_wall_displacement(self, wall, d, reproject=False):
        self._keep = self._dev(d, (self.nz, self.nx))
        lbm_set_wall_displacement(self.ctx, wall, self._keep, reproject)

    def set_wall_velocity(self, wall, v):
        self._keep_v = self._dev(v, (self.nz, self.nx, 3))
        lbm_set_wall_velocity(self.ctx, wall, self._keep_v)

    def set_plate(self, jp, i0, i1):
        """Interior plate between fluid rows jp-1 and jp over columns i0..i1
        (jp = 0 removes it); before the state is set."""
        lbm_set_plate(self.ctx, jp, i0, i1)

    def set_open_x(self, uin):
        """Open ends in x with the Cartesian inlet velocity [nz, H, 3] (None:
        periodic x again); before the state."""
        self._keep_in = self._dev(uin, (self.nz, self.H, 3))
        lbm_set_open_x(self.ctx, self._keep_in)

    def set_plate_displacement(self, d, reproject=False):
        self._keep_p = self._dev(d, (self.nz, self.nx))
        lbm_set_plate_displacement(self.ctx, self._keep_p, reproject)

    def set_plate_velocity(self, v):
        self._keep_pv = self._dev(v, (self.nz, self.nx, 3))
        lbm_set_plate_velocity(self.ctx, self._keep_pv)

    def plate_force(self, per_column=False):
        tot = torch.empty(3, dtype=torch.float64, device=self.device)
        pc = torch.empty((self.nz, self.nx, 3), dtype=torch.float64, device=self.device) if per_column else None
        lbm_plate_force(self.ctx, tot, pc)
        return (tot, pc) if per_column else tot

    def init_equilibrium(self, rho=None, ucart=None):
        r = self._dev(rho, self.fluid_shape)
        u = self._dev(ucart, (3,) + self.fluid_shape)
        lbm_init_equilibrium(self.ctx, r, u)
        self.stream.synchronize()

    def set_populations(self, f):
        t = self._dev(f, (19,) + self.fluid_shape)
        lbm_set_populations(self.ctx, t)
        self.stream.synchronize()

    def populations(self):
        out = torch.empty((19,) + self.fluid_shape, dtype=torch.float64, device=self.device)
        lbm_get_populations(self.ctx, out)
        return out

    def history(self):
        out = torch.empty((10,) + self.fluid_shape, dtype=torch.float64, device=self.device)
        lbm_get_history(self.ctx, out)
        return out

    def geometry(self):
        geo = torch.empty((28,) + self.fluid_shape, dtype=torch.float64, device=self.device)
        jac = torch.empty((9,) + self.fluid_shape, dtype=torch.float64, device=self.device)
        lbm_get_geometry(self.ctx, geo, jac)
        return geo, jac

    def step(self, n=1):
        lbm_step(self.ctx, n)

    def moments(self, cartesian=False):
        rho = torch.empty(self.fluid_shape, dtype=torch.float64, device=self.device)
        u = torch.empty((3,) + self.fluid_shape, dtype=torch.float64, device=self.device)
        lbm_moments(self.ctx, rho, u, cartesian)
        return rho, u

    def wall_force(self, wall, per_node=False, method=LBM_FORCE_STRESS):
        tot = torch.empty(3, dtype=torch.float64, device=self.device)
        pn = torch.empty((self.nz, self.nx, 3), dtype=torch.float64, device=self.device) if per_node else None
        lbm_wall_force(self.ctx, wall, tot, pn, method)
        return (tot, pn) if per_node else tot

    def couple(self, wall, disp, vcart, n):
        """One coupling interval (lbm_couple): new wall shape (or None),
        wall velocity (or None = at rest), n steps; returns the total and
        per-column force of the fluid on the wall."""
        self._keep = self._dev(disp, (self.nz, self.nx))
        self._keep_v = self._dev(vcart, (self.nz, self.nx, 3))
        tot = torch.empty(3, dtype=torch.float64, device=self.device)
        pn = torch.empty((self.nz, self.nx, 3), dtype=torch.float64, device=self.device)
        lbm_couple(self.ctx, wall, self._keep, self._keep_v, n, tot, pn)
        return tot, pn

    def sync(self):
        lbm_sync(self.ctx)

    def forward_record(self, K, wall=LBM_WALL_YMAX):
        """Run K steps from the current state, keeping checkpoints for
        backward(); returns the wall forces of states 1..K, [K, 3]."""
        forces = torch.empty((K, 3), dtype=torch.float64, device=self.device)
        lbm_forward_record(self.ctx, K, self.ckpt_every, wall, forces)
        self.recordings += 1
        return forces

    def backward(self, dLdF, need_disp=True, need_chart=False, need_f0=True):
        """Adjoint of the last forward_record for dL/dF [K, 3]: returns
        (dL/d top-wall displacement [nz, nx], dL/d chart [3, nz, ny, nx],
        dL/d f0 [19, nz, H, nx]); entries not asked for are None."""
        if not self.adjoint_K:
            raise ValueError("backward needs a solver created with adjoint_K > 0")
        # the library reads K x 3 doubles: a tensor of another size is refused here
        g = self._dev(dLdF)
        if g.numel() != 3 * self.adjoint_K:
            raise ValueError(f"dL/dF must hold [{self.adjoint_K}, 3] values, got {tuple(g.shape)}")
        g = g.reshape(self.adjoint_K, 3)
        gd = torch.empty((self.nz, self.nx), dtype=torch.float64, device=self.device) if need_disp else None
        gc = torch.empty((3, self.nz, self.ny, self.nx), dtype=torch.float64, device=self.device) if need_chart else None
        gf = torch.empty((19,) + self.fluid_shape, dtype=torch.float64, device=self.device) if need_f0 else None
        lbm_backward(self.ctx, g, gd, gc, gf)
        return gd, gc, gf


def _on_solver_stream(fn):
    """Run a Solver method with the context's stream current, ordered after
    the caller's stream (inputs it made are ready) and before it (outputs are
    ready to it); a no-op when the context uses the caller's stream."""

    @functools.wraps(fn)
    def run(self, *args, **kwargs):
        caller = torch.cuda.current_stream(self.device)
        if caller == self.stream:
            return fn(self, *args, **kwargs)
        self.stream.wait_stream(caller)
        with torch.cuda.stream(self.stream):
            out = fn(self, *args, **kwargs)
        caller.wait_stream(self.stream)
        return out

    return run


for _name, _fn in list(vars(Solver).items()):
    if callable(_fn) and not _name.startswith("_"):
        setattr(Solver, _name, _on_solver_stream(_fn))


class WallForceFn(torch.autograd.Function):
    """forces[K, 3] = wall forces of states 1..K after setting the top-wall
    displacement d [nz, nx] and the initial populations f0 [19, nz, H, nx] on
    `solver` (FP64; walls at rest or moving with the velocities set on it).
    backward returns (dL/dd, dL/df0); f0 is an independent input (its forcing
    history is recomputed from it).  The solver keeps one recording: backward
    raises if another forward_record ran on it since this forward."""

    @staticmethod
    def forward(ctx, d, f0, solver, K, wall=LBM_WALL_YMAX):
        solver.set_wall_displacement(LBM_WALL_YMAX, d.detach())
        solver.set_populations(f0.detach())
        forces = solver.forward_record(K, wall)
        ctx.solver = solver
        ctx.recording = solver.recordings
        return forces

    @staticmethod
    def backward(ctx, gF):
        if ctx.solver.recordings != ctx.recording:
            raise RuntimeError("WallForceFn: the solver recorded another trajectory since this forward; "
                               "its adjoint is no longer available")
        gd, _, gf = ctx.solver.backward(gF.contiguous(), need_disp=True, need_chart=False, need_f0=True)
        return gd, gf, None, None, None
