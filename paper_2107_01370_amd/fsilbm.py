"""Python binding of the C ABI in include/fsilbm.h (argument marshalling only).

Every numerical step runs in the HIP library ``lib/libfsilbm.so``; PyTorch is
used only to allocate the device workspace and to provide a HIP stream.
Functions keep the C names (``fsi_create``, ``fsi_step``, ...) and raise
:class:`FsiError` instead of returning a status.  :class:`Simulation` bundles
them for the common create / bind / init / step / query sequence.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FSILBM_LIB", os.path.join(_HERE, "lib", "libfsilbm.so"))

FSI_OK = 0
STATUS_NAMES = {0: "FSI_OK", -1: "FSI_E_ARG", -2: "FSI_E_MESH", -3: "FSI_E_CFL",
                -4: "FSI_E_STATE", -5: "FSI_E_HIP", -6: "FSI_E_NOMEM", -7: "FSI_E_UNBOUND"}
EXPORTED = ("fsi_create", "fsi_workspace_bytes", "fsi_bind_workspace", "fsi_init_equilibrium",
            "fsi_step", "fsi_step_noalloc", "fsi_synchronize", "fsi_get_step", "fsi_get_forces",
            "fsi_history_capacity", "fsi_get_body_state", "fsi_dump_macro",
            "fsi_get_populations", "fsi_set_populations", "fsi_state_bytes", "fsi_save",
            "fsi_load", "fsi_time_kernels", "fsi_set_coupling", "fsi_get_coupling_residual",
            "fsi_last_error", "fsi_destroy", "fsi_batch_create", "fsi_batch_workspace_bytes", "fsi_batch_bind_workspace",
            "fsi_batch_init_equilibrium", "fsi_batch_set_schedule", "fsi_batch_autotune",
            "fsi_batch_set_coupling", "fsi_batch_step", "fsi_batch_synchronize", "fsi_batch_get_forces",
            "fsi_batch_get_body_state", "fsi_batch_dump_macro", "fsi_batch_get_populations",
            "fsi_batch_time_kernels", "fsi_batch_nodes", "fsi_batch_last_error",
            "fsi_batch_destroy")


class FsiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class FluidParams(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("Pr", ctypes.c_double), ("mu", ctypes.c_double),
                ("rho_inf", ctypes.c_double), ("T_inf", ctypes.c_double),
                ("u_inf", ctypes.c_double * 2), ("dt", ctypes.c_double),
                ("storage", ctypes.c_int)]


class MeshDesc(ctypes.Structure):
    _fields_ = [("ni", ctypes.c_int), ("nj", ctypes.c_int), ("topo", ctypes.c_int),
                ("X", ctypes.POINTER(ctypes.c_double)), ("shift_i", ctypes.c_double * 2),
                ("shift_j", ctypes.c_double * 2), ("n_wake", ctypes.c_int),
                ("n_wall2", ctypes.c_int), ("n_elems", ctypes.c_int),
                ("elems", ctypes.POINTER(ctypes.c_int32)),
                ("elem_shifts", ctypes.POINTER(ctypes.c_int8)),
                ("n_wall_nodes", ctypes.c_int), ("wall_nodes", ctypes.POINTER(ctypes.c_int32)),
                ("n_far_nodes", ctypes.c_int), ("far_nodes", ctypes.POINTER(ctypes.c_int32))]


class BodyDesc(ctypes.Structure):
    _fields_ = [("dof", ctypes.c_int), ("m", ctypes.c_double), ("S_a", ctypes.c_double),
                ("I_a", ctypes.c_double), ("k_h", ctypes.c_double), ("k_a", ctypes.c_double),
                ("center", ctypes.c_double * 2), ("ea", ctypes.c_double * 2),
                ("r_rigid", ctypes.c_double), ("r_blend", ctypes.c_double),
                ("h0", ctypes.c_double), ("a0", ctypes.c_double), ("hd0", ctypes.c_double),
                ("ad0", ctypes.c_double), ("heave_amp", ctypes.c_double),
                ("heave_freq", ctypes.c_double), ("pitch_amp", ctypes.c_double),
                ("pitch_freq", ctypes.c_double), ("release_time", ctypes.c_double),
                ("blend_mode", ctypes.c_int), ("link", ctypes.c_int)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfsilbm.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FsiError(-5, f"HIP library not built: {path} (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    sig = {
        "fsi_create": (ctypes.c_int, [ctypes.POINTER(FluidParams), ctypes.POINTER(MeshDesc),
                                      ctypes.POINTER(BodyDesc), ctypes.c_int, P,
                                      ctypes.POINTER(P)]),
        "fsi_workspace_bytes": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_size_t)]),
        "fsi_bind_workspace": (ctypes.c_int, [P, P, ctypes.c_size_t]),
        "fsi_init_equilibrium": (ctypes.c_int, [P, dp, dp, dp, dp]),
        "fsi_step": (ctypes.c_int, [P, ctypes.c_int]),
        "fsi_step_noalloc": (ctypes.c_int, [P, ctypes.c_int]),
        "fsi_synchronize": (ctypes.c_int, [P]),
        "fsi_get_step": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_int64)]),
        "fsi_get_forces": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_int64, ctypes.c_int, dp]),
        "fsi_history_capacity": (ctypes.c_int64, []),
        "fsi_get_body_state": (ctypes.c_int, [P, ctypes.c_int, dp]),
        "fsi_dump_macro": (ctypes.c_int, [P, dp, dp, dp, dp]),
        "fsi_get_populations": (ctypes.c_int, [P, fp, fp]),
        "fsi_set_populations": (ctypes.c_int, [P, fp, fp]),
        "fsi_state_bytes": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_size_t)]),
        "fsi_save": (ctypes.c_int, [P, P, ctypes.c_size_t]),
        "fsi_load": (ctypes.c_int, [P, P, ctypes.c_size_t]),
        "fsi_time_kernels": (ctypes.c_int, [P, ctypes.c_int, dp]),
        "fsi_set_coupling": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_double]),
        "fsi_get_coupling_residual": (ctypes.c_int, [P, ctypes.c_int, dp]),
        "fsi_batch_set_coupling": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_double]),
        "fsi_last_error": (ctypes.c_char_p, [P]),
        "fsi_destroy": (None, [P]),
        "fsi_batch_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(FluidParams),
                                            ctypes.POINTER(MeshDesc), ctypes.POINTER(BodyDesc),
                                            ctypes.POINTER(ctypes.c_int), P, ctypes.POINTER(P)]),
        "fsi_batch_workspace_bytes": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_size_t)]),
        "fsi_batch_bind_workspace": (ctypes.c_int, [P, P, ctypes.c_size_t]),
        "fsi_batch_init_equilibrium": (ctypes.c_int, [P, ctypes.c_int, dp, dp, dp, dp]),
        "fsi_batch_set_schedule": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
        "fsi_batch_autotune": (ctypes.c_int, [P, ctypes.c_int, dp]),
        "fsi_batch_step": (ctypes.c_int, [P, ctypes.c_int]),
        "fsi_batch_synchronize": (ctypes.c_int, [P]),
        "fsi_batch_get_forces": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                                ctypes.c_int, dp]),
        "fsi_batch_get_body_state": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_int, dp]),
        "fsi_batch_dump_macro": (ctypes.c_int, [P, ctypes.c_int, dp, dp, dp, dp]),
        "fsi_batch_get_populations": (ctypes.c_int, [P, ctypes.c_int, fp, fp]),
        "fsi_batch_time_kernels": (ctypes.c_int, [P, ctypes.c_int, dp]),
        "fsi_batch_nodes": (ctypes.c_int64, [P]),
        "fsi_batch_last_error": (ctypes.c_char_p, [P]),
        "fsi_batch_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(ctx, status):
    if status != FSI_OK:
        msg = _lib.fsi_last_error(ctx).decode() if ctx else ""
        raise FsiError(status, msg)


def _dptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _f64(a, shape):
    if a is None:
        return None
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), shape))
    return a


# ---- thin wrappers with the C names ------------------------------------------

def _fluid_struct(fluid):
    return FluidParams(fluid.gamma, fluid.Pr, fluid.mu, fluid.rho_inf, fluid.T_inf,
                       (ctypes.c_double * 2)(*fluid.u_inf), fluid.dt, int(fluid.storage))


def _mesh_struct(mesh):
    """Returns (MeshDesc, arrays that must outlive the call)."""
    X = np.ascontiguousarray(mesh.interleaved(), dtype=np.float64)
    md = MeshDesc(mesh.ni, mesh.nj, mesh.topo, X.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                  (ctypes.c_double * 2)(*mesh.shift_i), (ctypes.c_double * 2)(*mesh.shift_j),
                  int(getattr(mesh, "n_wake", 0)), int(getattr(mesh, "n_wall2", 0)))
    keep = (X,)
    if getattr(mesh, "elems", None) is not None:
        el = np.ascontiguousarray(mesh.elems, dtype=np.int32)
        sh = np.ascontiguousarray(mesh.shifts, dtype=np.int8)
        md.n_elems = el.shape[0]
        md.elems = el.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        md.elem_shifts = sh.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
        keep = (X, el, sh)
        for name in ("wall_nodes", "far_nodes"):
            v = getattr(mesh, name, None)
            if v is not None and len(v):
                a = np.ascontiguousarray(v, dtype=np.int32)
                setattr(md, "n_" + name, a.size)
                setattr(md, name, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
                keep = keep + (a,)
    return md, keep


def _body_struct(b):
    return BodyDesc(int(b.dof), b.m, b.S_a, b.I_a, b.k_h, b.k_a,
                    (ctypes.c_double * 2)(*b.center), (ctypes.c_double * 2)(*b.ea),
                    b.r_rigid, b.r_blend, b.h0, b.a0, b.hd0, b.ad0, b.heave_amp,
                    b.heave_freq, b.pitch_amp, b.pitch_freq,
                    float(getattr(b, "release_time", 0.0)), int(getattr(b, "blend_mode", 0)),
                    int(getattr(b, "link", -1)))


def fsi_create(fluid, mesh, bodies=(), stream_handle=None):
    """fluid: synth.FluidParams-like; mesh: synth.MeshSpec-like; bodies: list of
    BodyParams-like (0 or 1; 2 on a twin O-grid).  Returns the context handle."""
    lib = load_library()
    fp = _fluid_struct(fluid)
    md, X = _mesh_struct(mesh)
    arr = (BodyDesc * max(1, len(bodies)))()
    for k, b in enumerate(bodies):
        arr[k] = _body_struct(b)
    ctx = ctypes.c_void_p()
    st = lib.fsi_create(ctypes.byref(fp), ctypes.byref(md), arr, len(bodies),
                        ctypes.c_void_p(stream_handle or 0), ctypes.byref(ctx))
    del X
    if st != FSI_OK:
        msg = lib.fsi_last_error(ctx).decode() if ctx.value else ""
        if ctx.value:
            lib.fsi_destroy(ctx)
        raise FsiError(st, msg)
    return ctx


def fsi_workspace_bytes(ctx):
    n = ctypes.c_size_t()
    _check(ctx, _lib.fsi_workspace_bytes(ctx, ctypes.byref(n)))
    return n.value


def fsi_bind_workspace(ctx, dev_ptr, nbytes):
    _check(ctx, _lib.fsi_bind_workspace(ctx, ctypes.c_void_p(dev_ptr), nbytes))


def fsi_init_equilibrium(ctx, shape, rho=None, ux=None, uy=None, T=None):
    arrs = [_f64(a, shape) for a in (rho, ux, uy, T)]
    _check(ctx, _lib.fsi_init_equilibrium(ctx, *[_dptr(a) for a in arrs]))


def fsi_step(ctx, nsteps):
    _check(ctx, _lib.fsi_step(ctx, int(nsteps)))


def fsi_step_noalloc(ctx, nsteps):
    _check(ctx, _lib.fsi_step_noalloc(ctx, int(nsteps)))


def fsi_synchronize(ctx):
    _check(ctx, _lib.fsi_synchronize(ctx))


def fsi_get_step(ctx):
    n = ctypes.c_int64()
    _check(ctx, _lib.fsi_get_step(ctx, ctypes.byref(n)))
    return n.value


def fsi_get_forces(ctx, first, count, body=0):
    out = np.zeros((count, 6), dtype=np.float64)
    _check(ctx, _lib.fsi_get_forces(ctx, body, int(first), int(count), _dptr(out)))
    return out


def fsi_history_capacity():
    return int(load_library().fsi_history_capacity())


def fsi_get_body_state(ctx, body=0):
    out = np.zeros(4, dtype=np.float64)
    _check(ctx, _lib.fsi_get_body_state(ctx, body, _dptr(out)))
    return out


def fsi_dump_macro(ctx, shape):
    outs = [np.empty(shape, dtype=np.float64) for _ in range(4)]
    _check(ctx, _lib.fsi_dump_macro(ctx, *[_dptr(o) for o in outs]))
    return tuple(outs)


def fsi_get_populations(ctx, shape):
    f = np.empty((9,) + tuple(shape), dtype=np.float32)
    g = np.empty((9,) + tuple(shape), dtype=np.float32)
    _check(ctx, _lib.fsi_get_populations(ctx, _fptr(f), _fptr(g)))
    return f, g


def fsi_set_populations(ctx, f, g):
    f = np.ascontiguousarray(f, dtype=np.float32)
    g = np.ascontiguousarray(g, dtype=np.float32)
    _check(ctx, _lib.fsi_set_populations(ctx, _fptr(f), _fptr(g)))


def fsi_state_bytes(ctx):
    n = ctypes.c_size_t()
    _check(ctx, _lib.fsi_state_bytes(ctx, ctypes.byref(n)))
    return n.value


def fsi_save(ctx):
    buf = ctypes.create_string_buffer(fsi_state_bytes(ctx))
    _check(ctx, _lib.fsi_save(ctx, ctypes.cast(buf, ctypes.c_void_p), len(buf)))
    return bytes(buf.raw)


def fsi_load(ctx, data: bytes):
    buf = ctypes.create_string_buffer(data, len(data))
    _check(ctx, _lib.fsi_load(ctx, ctypes.cast(buf, ctypes.c_void_p), len(data)))


def fsi_time_kernels(ctx, reps):
    """Mean ms per launch of (collide-stream, wall targets, wall Grad/traction, body)."""
    out = np.zeros(4, dtype=np.float64)
    _check(ctx, _lib.fsi_time_kernels(ctx, int(reps), _dptr(out)))
    return out


def fsi_set_coupling(ctx, subiterations, relaxation=1.0):
    _check(ctx, _lib.fsi_set_coupling(ctx, int(subiterations), float(relaxation)))


def fsi_get_coupling_residual(ctx, body=0):
    out = np.zeros(1, dtype=np.float64)
    _check(ctx, _lib.fsi_get_coupling_residual(ctx, int(body), _dptr(out)))
    return float(out[0])


def fsi_last_error(ctx):
    return _lib.fsi_last_error(ctx).decode()


def fsi_destroy(ctx):
    if ctx:
        _lib.fsi_destroy(ctx)


# ---- batches ---------------------------------------------------------------------

def _bcheck(b, status):
    if status != FSI_OK:
        msg = _lib.fsi_batch_last_error(b).decode() if b else ""
        raise FsiError(status, msg)


def fsi_batch_create(cases, stream_handle=None):
    """cases: sequence of (fluid, mesh, bodies); the bodies of all instances
    go to the library back to back."""
    lib = load_library()
    n = len(cases)
    fl = (FluidParams * n)()
    ms = (MeshDesc * n)()
    nb = (ctypes.c_int * n)()
    all_bodies = [b for (_, _, bodies) in cases for b in bodies]
    bd = (BodyDesc * max(1, len(all_bodies)))()
    for q, b in enumerate(all_bodies):
        bd[q] = _body_struct(b)
    keep = []
    for k, (fluid, mesh, bodies) in enumerate(cases):
        fl[k] = _fluid_struct(fluid)
        md, X = _mesh_struct(mesh)
        keep.append(X)
        ms[k] = md
        nb[k] = len(bodies)
    b = ctypes.c_void_p()
    st = lib.fsi_batch_create(n, fl, ms, bd, nb, ctypes.c_void_p(stream_handle or 0),
                              ctypes.byref(b))
    del keep
    if st != FSI_OK:
        msg = lib.fsi_batch_last_error(b).decode() if b.value else ""
        if b.value:
            lib.fsi_batch_destroy(b)
        raise FsiError(st, msg)
    return b


def fsi_batch_workspace_bytes(b):
    n = ctypes.c_size_t()
    _bcheck(b, _lib.fsi_batch_workspace_bytes(b, ctypes.byref(n)))
    return n.value


def fsi_batch_bind_workspace(b, dev_ptr, nbytes):
    _bcheck(b, _lib.fsi_batch_bind_workspace(b, ctypes.c_void_p(dev_ptr), nbytes))


def fsi_batch_init_equilibrium(b, k, shape, rho=None, ux=None, uy=None, T=None):
    arrs = [_f64(a, shape) for a in (rho, ux, uy, T)]
    _bcheck(b, _lib.fsi_batch_init_equilibrium(b, int(k), *[_dptr(a) for a in arrs]))


# default tile shape of a batch's instances (32 x 16; see fsi_batch_set_schedule)
DEFAULT_SHAPE = 0


def fsi_batch_set_schedule(b, grid, order, shape=DEFAULT_SHAPE):
    _bcheck(b, _lib.fsi_batch_set_schedule(b, int(grid), int(order), int(shape)))


def fsi_batch_autotune(b, reps):
    """Returns (grid, order, shape, ms per collision-streaming launch) of the
    fastest schedule."""
    out = np.zeros(4, dtype=np.float64)
    _bcheck(b, _lib.fsi_batch_autotune(b, int(reps), _dptr(out)))
    return int(out[0]), int(out[1]), int(out[2]), float(out[3])


def fsi_batch_set_coupling(b, subiterations, relaxation=1.0):
    _bcheck(b, _lib.fsi_batch_set_coupling(b, int(subiterations), float(relaxation)))


def fsi_batch_step(b, nsteps):
    _bcheck(b, _lib.fsi_batch_step(b, int(nsteps)))


def fsi_batch_synchronize(b):
    _bcheck(b, _lib.fsi_batch_synchronize(b))


def fsi_batch_get_forces(b, k, first, count, body=0):
    out = np.zeros((count, 6), dtype=np.float64)
    _bcheck(b, _lib.fsi_batch_get_forces(b, int(k), int(body), int(first), int(count),
                                         _dptr(out)))
    return out


def fsi_batch_get_body_state(b, k, body=0):
    out = np.zeros(4, dtype=np.float64)
    _bcheck(b, _lib.fsi_batch_get_body_state(b, int(k), int(body), _dptr(out)))
    return out


def fsi_batch_dump_macro(b, k, shape):
    outs = [np.empty(shape, dtype=np.float64) for _ in range(4)]
    _bcheck(b, _lib.fsi_batch_dump_macro(b, int(k), *[_dptr(o) for o in outs]))
    return tuple(outs)


def fsi_batch_get_populations(b, k, shape):
    f = np.empty((9,) + tuple(shape), dtype=np.float32)
    g = np.empty((9,) + tuple(shape), dtype=np.float32)
    _bcheck(b, _lib.fsi_batch_get_populations(b, int(k), _fptr(f), _fptr(g)))
    return f, g


def fsi_batch_time_kernels(b, reps):
    out = np.zeros(4, dtype=np.float64)
    _bcheck(b, _lib.fsi_batch_time_kernels(b, int(reps), _dptr(out)))
    return out


def fsi_batch_nodes(b):
    return int(_lib.fsi_batch_nodes(b))


def fsi_batch_last_error(b):
    return _lib.fsi_batch_last_error(b).decode()


def fsi_batch_destroy(b):
    if b:
        _lib.fsi_batch_destroy(b)


# ---- convenience wrapper -------------------------------------------------------

class Simulation:
    """One mesh + (optional) body on one GPU.

    ``torch`` provides the device workspace and a dedicated HIP stream (default
    priority); every step runs in the library's kernels.
    """

    def __init__(self, mesh, fluid, bodies=(), device="cuda:0"):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.shape = (mesh.nj, mesh.ni)
        self.mesh = mesh
        self.stream = torch.cuda.Stream(device=self.device)
        self.ctx = fsi_create(fluid, mesh, list(bodies), self.stream.cuda_stream)
        try:
            nbytes = fsi_workspace_bytes(self.ctx)
            # over-allocate by 256 bytes so the workspace can be 256-byte aligned
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            self.ws_ptr = (base + 255) & ~255
            fsi_bind_workspace(self.ctx, self.ws_ptr, nbytes)
        except Exception:
            fsi_destroy(self.ctx)
            self.ctx = None
            raise

    def init_equilibrium(self, rho=None, ux=None, uy=None, T=None):
        fsi_init_equilibrium(self.ctx, self.shape, rho, ux, uy, T)

    def step(self, nsteps=1):
        fsi_step(self.ctx, nsteps)

    def step_noalloc(self, nsteps=1):
        fsi_step_noalloc(self.ctx, nsteps)

    def synchronize(self):
        fsi_synchronize(self.ctx)

    def step_count(self):
        return fsi_get_step(self.ctx)

    def forces(self, first, count, body=0):
        return fsi_get_forces(self.ctx, first, count, body)

    def body_state(self, body=0):
        return fsi_get_body_state(self.ctx, body)

    def set_coupling(self, subiterations, relaxation=1.0):
        fsi_set_coupling(self.ctx, subiterations, relaxation)

    def coupling_residual(self, body=0):
        return fsi_get_coupling_residual(self.ctx, body)

    def macro(self):
        return fsi_dump_macro(self.ctx, self.shape)

    def populations(self):
        return fsi_get_populations(self.ctx, self.shape)

    def set_populations(self, f, g):
        fsi_set_populations(self.ctx, f, g)

    def save(self):
        return fsi_save(self.ctx)

    def load(self, data):
        fsi_load(self.ctx, data)

    def time_kernels(self, reps=20):
        return fsi_time_kernels(self.ctx, reps)

    def close(self):
        # fsi_destroy drains the stream before the workspace can be released
        if self.ctx:
            fsi_destroy(self.ctx)
            self.ctx = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent instances on one GPU, advanced by one launch per kernel.

    ``cases``: sequence of objects with ``mesh``, ``fluid`` and ``bodies``
    (``synth.Case``), or of (fluid, mesh, bodies) tuples.
    """

    def __init__(self, cases, device="cuda:0"):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        triples = [c if isinstance(c, tuple) else (c.fluid, c.mesh, list(c.bodies)) for c in cases]
        self.shapes = [(m.nj, m.ni) for _, m, _ in triples]
        self.stream = torch.cuda.Stream(device=self.device)
        self.b = fsi_batch_create(triples, self.stream.cuda_stream)
        try:
            nbytes = fsi_batch_workspace_bytes(self.b)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self.ws_ptr = (self.workspace.data_ptr() + 255) & ~255
            fsi_batch_bind_workspace(self.b, self.ws_ptr, nbytes)
        except Exception:
            fsi_batch_destroy(self.b)
            self.b = None
            raise

    def __len__(self):
        return len(self.shapes)

    def nodes(self):
        return fsi_batch_nodes(self.b)

    def init_equilibrium(self, k, rho=None, ux=None, uy=None, T=None):
        fsi_batch_init_equilibrium(self.b, k, self.shapes[k], rho, ux, uy, T)

    def set_schedule(self, grid, order, shape=DEFAULT_SHAPE):
        fsi_batch_set_schedule(self.b, grid, order, shape)

    def autotune(self, reps=5):
        return fsi_batch_autotune(self.b, reps)

    def set_coupling(self, subiterations, relaxation=1.0):
        fsi_batch_set_coupling(self.b, subiterations, relaxation)

    def step(self, nsteps=1):
        fsi_batch_step(self.b, nsteps)

    def synchronize(self):
        fsi_batch_synchronize(self.b)

    def forces(self, k, first, count, body=0):
        return fsi_batch_get_forces(self.b, k, first, count, body)

    def body_state(self, k, body=0):
        return fsi_batch_get_body_state(self.b, k, body)

    def macro(self, k):
        return fsi_batch_dump_macro(self.b, k, self.shapes[k])

    def populations(self, k):
        return fsi_batch_get_populations(self.b, k, self.shapes[k])

    def time_kernels(self, reps=20):
        return fsi_batch_time_kernels(self.b, reps)

    def close(self):
        if self.b:
            fsi_batch_destroy(self.b)
            self.b = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
