"""ctypes binding of libdg.so: the functions of include/dg.h under the same
names, taking torch CUDA tensors (or raw device pointers) for device arrays.

Argument marshalling only: tensors are checked for device, dtype, contiguity
and size, then their data pointers and the current torch stream are handed to
the C ABI.  Every computation runs in the library's HIP kernels; there is no
CPU or PyTorch fallback, and importing this module fails if the library is
missing.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2006_15698_amd.build`")

# torch brings its own HIP runtime (libamdhip64.so under torch/lib, soname
# libamdhip64.so.7).  Loading torch first makes the dynamic loader resolve
# libdg.so's libamdhip64.so.7 to that same runtime; loading libdg.so first
# would map a second HIP/HSA runtime into the process.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

DG_OK = 0
DG_EINVAL = -1
DG_EUNSUPPORTED = -2
DG_EHIP = -3
DG_EALIAS = -4
DG_ENONPHYSICAL = -5
DG_EWORKSPACE = -6
DG_FP64 = 0
DG_FP32_MFMA = 1
DG_VOLUME_STANDARD = 0
DG_VOLUME_KEP = 1
DG_OPT_EXCHANGE = 1
DG_OPT_XCD_REMAP = 2
DG_OPT_ORDER = 3
DG_OPT_PENCIL_X = 4
DG_OPT_PENCIL_Z = 5
DG_EXCHANGE_TRACES = 0
DG_EXCHANGE_NEIGHBOUR = 1
DG_ORDER_LINEAR = 0
DG_ORDER_PENCIL = 1
DG_OPT_BATCH_LAUNCH = 6
DG_OPT_VISC_FUSED = 7
DG_BATCH_PERSISTENT = 0
DG_BATCH_PER_DEGREE = 1
OPTION_NAMES = {DG_OPT_EXCHANGE: "exchange", DG_OPT_XCD_REMAP: "xcd_remap", DG_OPT_ORDER: "order",
                DG_OPT_PENCIL_X: "pencil_x", DG_OPT_PENCIL_Z: "pencil_z", DG_OPT_VISC_FUSED: "visc_fused"}
BATCH_OPTION_NAMES = {DG_OPT_XCD_REMAP: "xcd_remap", DG_OPT_ORDER: "order", DG_OPT_PENCIL_X: "pencil_x",
                      DG_OPT_PENCIL_Z: "pencil_z", DG_OPT_BATCH_LAUNCH: "batch_launch"}

ERROR_NAMES = {DG_EINVAL: "DG_EINVAL", DG_EUNSUPPORTED: "DG_EUNSUPPORTED", DG_EHIP: "DG_EHIP",
               DG_EALIAS: "DG_EALIAS", DG_ENONPHYSICAL: "DG_ENONPHYSICAL",
               DG_EWORKSPACE: "DG_EWORKSPACE"}

_vp, _i, _d, _sz, _i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "dg_create": (_vp, [_i, _i, _i, _i, _d]),
    "dg_destroy": (None, [_vp]),
    "dg_last_error": (ctypes.c_char_p, []),
    "dg_set_domain": (_i, [_vp, _d, _d, _d]),
    "dg_set_stream": (_i, [_vp, _vp]),
    "dg_set_precision": (_i, [_vp, _i]),
    "dg_set_viscosity": (_i, [_vp, _d, _d]),
    "dg_set_volume_form": (_i, [_vp, _i]),
    "dg_workspace_bytes": (_sz, [_vp]),
    "dg_set_workspace": (_i, [_vp, _vp, _sz]),
    "dg_num_dof": (_i64, [_vp]),
    "dg_quadrature": (_i, [_i, _dp, _dp]),
    "dg_rhs": (_i, [_vp, _vp, _vp]),
    "dg_rk_stage": (_i, [_vp, _i, _vp, _vp, _d]),
    "dg_rk_step": (_i, [_vp, _vp, _vp, _d]),
    "dg_rk_steps": (_i, [_vp, _vp, _vp, _d, _i]),
    "dg_rk_graph_steps": (_i, [_vp, _vp, _vp, _d, _i]),
    "dg_rk_steps_noalloc": (_i, [_vp, _vp, _vp, _d, _i]),
    "dg_rhs_vjp": (_i, [_vp, _vp, _vp, _vp]),
    "dg_rk_stage_vjp": (_i, [_vp, _i, _vp, _vp, _vp, _d]),
    "dg_kinetic_energy_grad": (_i, [_vp, _vp, _vp]),
    "dg_recip_sqrt": (_i, [_vp, _vp, _vp, _i64, _vp]),
    "dg_integrals": (_i, [_vp, _vp, _dp]),
    "dg_max_wavespeed": (_i, [_vp, _vp, _dp]),
    "dg_check_state": (_i, [_vp, _vp]),
    "dg_batch_create": (_vp, [_i, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), _dp, _d]),
    "dg_batch_destroy": (None, [_vp]),
    "dg_batch_set_stream": (_i, [_vp, _vp]),
    "dg_batch_set_precision": (_i, [_vp, _i]),
    "dg_batch_set_tile": (_i, [_vp, _i, _i]),
    "dg_batch_set_option": (_i, [_vp, _i, _i]),
    "dg_batch_get_option": (_i, [_vp, _i, ctypes.POINTER(ctypes.c_int)]),
    "dg_batch_tile_options": (_i, [_i, ctypes.POINTER(ctypes.c_int), _i]),
    "dg_batch_offset": (_i64, [_vp, _i]),
    "dg_batch_workspace_bytes": (_sz, [_vp]),
    "dg_batch_set_workspace": (_i, [_vp, _vp, _sz]),
    "dg_batch_set_dt": (_i, [_vp, _dp]),
    "dg_batch_rhs": (_i, [_vp, _vp, _vp]),
    "dg_batch_rk_steps": (_i, [_vp, _vp, _vp, _i]),
    "dg_batch_graph_steps": (_i, [_vp, _vp, _vp, _i]),
    "dg_varp_create": (_vp, [_i, _i, _i, ctypes.POINTER(ctypes.c_int), _dp, _d]),
    "dg_varp_create_refined": (_vp, [_i, _i, _i, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), _dp,
                                     _d]),
    "dg_varp_num_elements": (_i64, [_vp]),
    "dg_varp_destroy": (None, [_vp]),
    "dg_varp_set_stream": (_i, [_vp, _vp]),
    "dg_varp_num_dof": (_i64, [_vp]),
    "dg_varp_offset": (_i64, [_vp, _i64]),
    "dg_varp_workspace_bytes": (_sz, [_vp]),
    "dg_varp_set_workspace": (_i, [_vp, _vp, _sz]),
    "dg_varp_rhs": (_i, [_vp, _vp, _vp]),
    "dg_varp_rk_steps": (_i, [_vp, _vp, _vp, _d, _i]),
    "dg_varp_set_timing": (_i, [_vp, _i]),
    "dg_varp_timing_read": (_i, [_vp, _dp, ctypes.POINTER(ctypes.c_int64)]),
    "dg_set_option": (_i, [_vp, _i, _i]),
    "dg_get_option": (_i, [_vp, _i, ctypes.POINTER(ctypes.c_int)]),
    "dg_set_timing": (_i, [_vp, _i]),
    "dg_timing_read": (_i, [_vp, _dp, ctypes.POINTER(ctypes.c_int64)]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class DGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def dg_last_error():
    return _lib.dg_last_error().decode()


def _check(rc):
    if rc != DG_OK:
        raise DGError(rc, dg_last_error())
    return rc


def _ptr(x, nd=None):
    """Device pointer of a torch CUDA tensor (float64, contiguous, numel nd)
    or of a raw integer address."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    import torch
    if not isinstance(x, torch.Tensor):
        raise TypeError("expected a torch tensor or a device address")
    if not x.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not x.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if nd is not None:
        if x.dtype != torch.float64:
            raise ValueError("state arrays are float64")
        if x.numel() != nd:
            raise ValueError(f"tensor has {x.numel()} elements, expected {nd}")
    return x.data_ptr()


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---- the C ABI under the same names ---------------------------------------
def dg_create(nx, ny, nz, p, gamma=1.4):
    ctx = _lib.dg_create(int(nx), int(ny), int(nz), int(p), float(gamma))
    if not ctx:
        raise DGError(DG_EINVAL, dg_last_error())
    return ctx


def dg_destroy(ctx):
    _lib.dg_destroy(ctx)


def dg_set_domain(ctx, Lx, Ly, Lz):
    return _check(_lib.dg_set_domain(ctx, float(Lx), float(Ly), float(Lz)))


def dg_set_stream(ctx, stream=None):
    return _check(_lib.dg_set_stream(ctx, _stream_ptr(stream)))


def dg_set_precision(ctx, mode):
    return _check(_lib.dg_set_precision(ctx, int(mode)))


def dg_set_viscosity(ctx, mu, prandtl=0.72):
    return _check(_lib.dg_set_viscosity(ctx, float(mu), float(prandtl)))


def dg_set_volume_form(ctx, form):
    return _check(_lib.dg_set_volume_form(ctx, int(form)))


def dg_set_option(ctx, key, value):
    return _check(_lib.dg_set_option(ctx, int(key), int(value)))


def dg_get_option(ctx, key):
    v = ctypes.c_int(0)
    _check(_lib.dg_get_option(ctx, int(key), ctypes.byref(v)))
    return v.value


def dg_workspace_bytes(ctx):
    return int(_lib.dg_workspace_bytes(ctx))


def dg_set_workspace(ctx, ws, nbytes=None):
    if nbytes is None:
        nbytes = ws.numel() * ws.element_size()
    return _check(_lib.dg_set_workspace(ctx, _ptr(ws), int(nbytes)))


def dg_num_dof(ctx):
    return int(_lib.dg_num_dof(ctx))


def dg_quadrature(p):
    n = p + 1
    xi = (ctypes.c_double * n)()
    w = (ctypes.c_double * n)()
    _check(_lib.dg_quadrature(int(p), xi, w))
    return np.array(xi[:]), np.array(w[:])


def _nd(ctx):
    return 5 * dg_num_dof(ctx)


def dg_rhs(ctx, Q, R):
    nd = _nd(ctx)
    return _check(_lib.dg_rhs(ctx, _ptr(Q, nd), _ptr(R, nd)))


def dg_rk_stage(ctx, s, Q, res, dt):
    nd = _nd(ctx)
    return _check(_lib.dg_rk_stage(ctx, int(s), _ptr(Q, nd), _ptr(res, nd), float(dt)))


def dg_rk_step(ctx, Q, res, dt):
    nd = _nd(ctx)
    return _check(_lib.dg_rk_step(ctx, _ptr(Q, nd), _ptr(res, nd), float(dt)))


def dg_rk_steps(ctx, Q, res, dt, nsteps):
    nd = _nd(ctx)
    return _check(_lib.dg_rk_steps(ctx, _ptr(Q, nd), _ptr(res, nd), float(dt), int(nsteps)))


def dg_rk_steps_noalloc(ctx, Q, res, dt, nsteps):
    nd = _nd(ctx)
    return _check(_lib.dg_rk_steps_noalloc(ctx, _ptr(Q, nd), _ptr(res, nd), float(dt), int(nsteps)))


DG_NOALLOC_MAX_BYTES = 128 << 20


def dg_rk_graph_steps(ctx, Q, res, dt, nsteps):
    nd = _nd(ctx)
    return _check(_lib.dg_rk_graph_steps(ctx, _ptr(Q, nd), _ptr(res, nd), float(dt), int(nsteps)))


def dg_rhs_vjp(ctx, Q, gR, gQ):
    nd = _nd(ctx)
    return _check(_lib.dg_rhs_vjp(ctx, _ptr(Q, nd), _ptr(gR, nd), _ptr(gQ, nd)))


def dg_rk_stage_vjp(ctx, s, Qs, gQ, gres, dt):
    nd = _nd(ctx)
    return _check(_lib.dg_rk_stage_vjp(ctx, int(s), _ptr(Qs, nd), _ptr(gQ, nd), _ptr(gres, nd), float(dt)))


def dg_kinetic_energy_grad(ctx, Q, gQ):
    nd = _nd(ctx)
    return _check(_lib.dg_kinetic_energy_grad(ctx, _ptr(Q, nd), _ptr(gQ, nd)))


def dg_recip_sqrt(x, r, s, stream=None):
    """r = 1/x, s = sqrt(x) elementwise with the kernels' own reciprocal and
    square root (float64 device tensors of equal size)."""
    n = x.numel()
    return _check(_lib.dg_recip_sqrt(_ptr(x, n), _ptr(r, n), _ptr(s, n), n, _stream_ptr(stream)))


def dg_integrals(ctx, Q):
    out = (ctypes.c_double * 6)()
    _check(_lib.dg_integrals(ctx, _ptr(Q, _nd(ctx)), out))
    return np.array(out[:])


def dg_max_wavespeed(ctx, Q):
    out = ctypes.c_double()
    _check(_lib.dg_max_wavespeed(ctx, _ptr(Q, _nd(ctx)), ctypes.byref(out)))
    return out.value


def dg_check_state(ctx, Q):
    """True if the state is physical; False on DG_ENONPHYSICAL."""
    rc = _lib.dg_check_state(ctx, _ptr(Q, _nd(ctx)))
    if rc == DG_ENONPHYSICAL:
        return False
    _check(rc)
    return True


TIMING_KINDS = ("trace", "stage", "rhs", "vjp", "reduce", "stage_first", "visc")


def dg_set_timing(ctx, on):
    return _check(_lib.dg_set_timing(ctx, 1 if on else 0))


def dg_timing_read(ctx):
    """{kind: (milliseconds, launches)} since timing was switched on."""
    ms = (ctypes.c_double * len(TIMING_KINDS))()
    cnt = (ctypes.c_int64 * len(TIMING_KINDS))()
    _check(_lib.dg_timing_read(ctx, ms, cnt))
    return {k: (ms[i], cnt[i]) for i, k in enumerate(TIMING_KINDS)}


# ---- batched meshes ----------------------------------------------------------
def dg_batch_create(n, p, L, gamma=1.4):
    """n: list of (nx, ny, nz); p: list of degrees; L: list of (Lx, Ly, Lz)."""
    count = len(p)
    na = (ctypes.c_int * (3 * count))(*[int(v) for t in n for v in t])
    pa = (ctypes.c_int * count)(*[int(v) for v in p])
    La = (ctypes.c_double * (3 * count))(*[float(v) for t in L for v in t])
    b = _lib.dg_batch_create(count, na, pa, La, float(gamma))
    if not b:
        raise DGError(DG_EINVAL, dg_last_error())
    return b


def dg_batch_destroy(b):
    _lib.dg_batch_destroy(b)


def dg_batch_set_stream(b, stream=None):
    return _check(_lib.dg_batch_set_stream(b, _stream_ptr(stream)))


def dg_batch_set_precision(b, mode):
    return _check(_lib.dg_batch_set_precision(b, int(mode)))


def dg_batch_set_tile(b, p, epb):
    return _check(_lib.dg_batch_set_tile(b, int(p), int(epb)))


def dg_batch_set_option(b, key, value):
    return _check(_lib.dg_batch_set_option(b, int(key), int(value)))


def dg_batch_get_option(b, key):
    v = ctypes.c_int(0)
    _check(_lib.dg_batch_get_option(b, int(key), ctypes.byref(v)))
    return v.value


def dg_batch_tile_options(p):
    out = (ctypes.c_int * 16)()
    k = _lib.dg_batch_tile_options(int(p), out, 16)
    return [out[i] for i in range(k)]


def dg_batch_offset(b, i):
    return int(_lib.dg_batch_offset(b, int(i)))


def dg_batch_workspace_bytes(b):
    return int(_lib.dg_batch_workspace_bytes(b))


def dg_batch_set_workspace(b, ws, nbytes=None):
    if nbytes is None:
        nbytes = ws.numel() * ws.element_size()
    return _check(_lib.dg_batch_set_workspace(b, _ptr(ws), int(nbytes)))


def dg_batch_set_dt(b, dt):
    arr = (ctypes.c_double * len(dt))(*[float(v) for v in dt])
    return _check(_lib.dg_batch_set_dt(b, arr))


def dg_batch_rhs(b, Q, R):
    return _check(_lib.dg_batch_rhs(b, _ptr(Q), _ptr(R)))


def dg_batch_rk_steps(b, Q, res, nsteps):
    return _check(_lib.dg_batch_rk_steps(b, _ptr(Q), _ptr(res), int(nsteps)))


def dg_batch_graph_steps(b, Q, res, nsteps):
    return _check(_lib.dg_batch_graph_steps(b, _ptr(Q), _ptr(res), int(nsteps)))


class Batch:
    """Independent periodic meshes advanced together on one GPU.  State is
    one flat float64 tensor; ``view(Q, i)`` is mesh i's block shaped
    [5, nz, ny, nx, N, N, N]."""

    def __init__(self, n, p, L, gamma=1.4, precision=DG_FP64, tiles=None, device=None):
        self.n = [tuple(int(v) for v in t) for t in n]
        self.p = [int(v) for v in p]
        self.L = [tuple(float(v) for v in t) for t in L]
        self.count = len(self.p)
        self.device = torch.device(device or "cuda")
        self.b = dg_batch_create(self.n, self.p, self.L, gamma)
        dg_batch_set_precision(self.b, precision)
        if tiles is None:
            from .tune import load_tiles
            tiles = load_tiles() or {}
        self.tiles = dict(tiles)
        for deg, epb in tiles.items():
            dg_batch_set_tile(self.b, deg, epb)
        self.offsets = [dg_batch_offset(self.b, i) for i in range(self.count + 1)]
        nbytes = dg_batch_workspace_bytes(self.b)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        _check(_lib.dg_batch_set_workspace(self.b, aligned, nbytes))

    def __del__(self):
        b = getattr(self, "b", None)
        # at interpreter exit the module's functions may already be gone
        if b and dg_batch_destroy is not None:
            dg_batch_destroy(b)
            self.b = None

    @property
    def total(self):
        return self.offsets[-1]

    def empty(self):
        return torch.empty(self.total, dtype=torch.float64, device=self.device)

    def view(self, Q, i):
        nx, ny, nz = self.n[i]
        N = self.p[i] + 1
        return Q[self.offsets[i]:self.offsets[i + 1]].view(5, nz, ny, nx, N, N, N)

    def pack(self, states):
        Q = self.empty()
        for i, st in enumerate(states):
            self.view(Q, i).copy_(st if isinstance(st, torch.Tensor) else torch.from_numpy(st))
        return Q

    def _s(self):
        dg_batch_set_stream(self.b, None)

    def set_option(self, key, value):
        """Work-list visiting order (DG_OPT_XCD_REMAP, DG_OPT_ORDER,
        DG_OPT_PENCIL_X, DG_OPT_PENCIL_Z) and launch form
        (DG_OPT_BATCH_LAUNCH); results are bitwise unchanged."""
        self._s()
        dg_batch_set_option(self.b, key, value)

    def options(self):
        return {name: dg_batch_get_option(self.b, k) for k, name in BATCH_OPTION_NAMES.items()}

    def set_dt(self, dt):
        self._s()
        dg_batch_set_dt(self.b, dt)

    def rhs(self, Q, out=None):
        out = self.empty() if out is None else out
        self._s()
        dg_batch_rhs(self.b, Q, out)
        return out

    def step(self, Q, res, nsteps=1, graph=False):
        self._s()
        if graph:
            dg_batch_graph_steps(self.b, Q, res, nsteps)
        else:
            dg_batch_rk_steps(self.b, Q, res, nsteps)


# ---- variable degree per element -------------------------------------------
def dg_varp_create(nx, ny, nz, degrees, L=(1.0, 1.0, 1.0), gamma=1.4):
    """degrees: E integers in element order e = (ez ny + ey) nx + ex."""
    deg = [int(v) for v in np.asarray(degrees).reshape(-1)]
    if len(deg) != nx * ny * nz:
        raise ValueError(f"{len(deg)} degrees for {nx * ny * nz} elements")
    da = (ctypes.c_int * len(deg))(*deg)
    La = (ctypes.c_double * 3)(*[float(v) for v in L])
    v = _lib.dg_varp_create(int(nx), int(ny), int(nz), da, La, float(gamma))
    if not v:
        raise DGError(DG_EINVAL, dg_last_error())
    return v


def dg_varp_create_refined(nx, ny, nz, refine, degrees, L=(1.0, 1.0, 1.0), gamma=1.4):
    """refine: nx ny nz values 0/1 in cell order c = (cz ny + cy) nx + cx;
    degrees: one per element, cell by cell, a refined cell's eight children
    in the order (kz, ky, kx)."""
    ref = [int(v) for v in np.asarray(refine).reshape(-1)]
    if len(ref) != nx * ny * nz:
        raise ValueError(f"{len(ref)} refinement flags for {nx * ny * nz} cells")
    deg = [int(v) for v in np.asarray(degrees).reshape(-1)]
    E = nx * ny * nz + 7 * sum(1 for r in ref if r)
    if len(deg) != E:
        raise ValueError(f"{len(deg)} degrees for {E} elements")
    ra = (ctypes.c_int * len(ref))(*ref)
    da = (ctypes.c_int * len(deg))(*deg)
    La = (ctypes.c_double * 3)(*[float(v) for v in L])
    v = _lib.dg_varp_create_refined(int(nx), int(ny), int(nz), ra, da, La, float(gamma))
    if not v:
        raise DGError(DG_EINVAL, dg_last_error())
    return v


def dg_varp_destroy(v):
    _lib.dg_varp_destroy(v)


def dg_varp_num_elements(v):
    return int(_lib.dg_varp_num_elements(v))


def dg_varp_set_stream(v, stream=None):
    return _check(_lib.dg_varp_set_stream(v, _stream_ptr(stream)))


def dg_varp_num_dof(v):
    return int(_lib.dg_varp_num_dof(v))


def dg_varp_offset(v, e):
    return int(_lib.dg_varp_offset(v, int(e)))


def dg_varp_workspace_bytes(v):
    return int(_lib.dg_varp_workspace_bytes(v))


def dg_varp_set_workspace(v, ws, nbytes=None):
    if nbytes is None:
        nbytes = ws.numel() * ws.element_size()
    return _check(_lib.dg_varp_set_workspace(v, _ptr(ws), int(nbytes)))


def dg_varp_rhs(v, Q, R):
    return _check(_lib.dg_varp_rhs(v, _ptr(Q), _ptr(R)))


def dg_varp_rk_steps(v, Q, res, dt, nsteps):
    return _check(_lib.dg_varp_rk_steps(v, _ptr(Q), _ptr(res), float(dt), int(nsteps)))


def dg_varp_set_timing(v, on):
    return _check(_lib.dg_varp_set_timing(v, int(on)))


DG_VARP_TIMING_SLOTS = 26


def dg_varp_timing_read(v):
    """{(p, mode): (ms, launches)} for the launches recorded since timing
    was switched on (mode 0 rhs, 1 stages 2..5, 2 first stage; both element
    sizes), "mortar": (ms, launches) for the kernel of the faces between
    degrees and "hanging" for the hanging-face kernel."""
    ms = (ctypes.c_double * DG_VARP_TIMING_SLOTS)()
    cnt = (ctypes.c_int64 * DG_VARP_TIMING_SLOTS)()
    _check(_lib.dg_varp_timing_read(v, ms, cnt))
    out = {(i // 3, i % 3): (ms[i], cnt[i]) for i in range(24) if cnt[i]}
    if cnt[24]:
        out["mortar"] = (ms[24], cnt[24])
    if cnt[25]:
        out["hanging"] = (ms[25], cnt[25])
    return out


class VariableDegree:
    """Periodic mesh of nx*ny*nz cells with a degree per element.  Without
    refine: one element per cell, degrees[ez, ey, ex] (0..7).  With refine
    (refine[cz, cy, cx] in {0, 1}): a refined cell is eight elements of half
    its size, elements cell by cell with a refined cell's children in the
    order (kz, ky, kx), and degrees one per element in that order.  State: a
    flat float64 tensor of 5 T values, field f at [f T, (f + 1) T), element
    e's nodes at offsets[e] .. offsets[e + 1]."""

    def __init__(self, n, degrees, L=(1.0, 1.0, 1.0), gamma=1.4, device=None, refine=None):
        self.nx, self.ny, self.nz = (int(v) for v in n)
        self.L = tuple(float(v) for v in L)
        self.gamma = float(gamma)
        self.device = torch.device(device or "cuda")
        if refine is None:
            self.refine = None
            self.deg = np.asarray(degrees, dtype=np.int64).reshape(self.nz, self.ny, self.nx)
            self.v = dg_varp_create(self.nx, self.ny, self.nz, self.deg, self.L, self.gamma)
        else:
            self.refine = np.asarray(refine, dtype=np.int64).reshape(self.nz, self.ny, self.nx)
            self.deg = np.asarray(degrees, dtype=np.int64).reshape(-1)
            self.v = dg_varp_create_refined(self.nx, self.ny, self.nz, self.refine, self.deg, self.L, self.gamma)
        self.T = dg_varp_num_dof(self.v)
        self.E = dg_varp_num_elements(self.v)
        self.offsets = [dg_varp_offset(self.v, e) for e in range(self.E + 1)]
        nbytes = dg_varp_workspace_bytes(self.v)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        _check(_lib.dg_varp_set_workspace(self.v, aligned, nbytes))

    def __del__(self):
        v = getattr(self, "v", None)
        if v and dg_varp_destroy is not None:
            dg_varp_destroy(v)
            self.v = None

    def num_dof(self):
        return self.T

    def empty(self):
        return torch.empty(5 * self.T, dtype=torch.float64, device=self.device)

    def _s(self):
        dg_varp_set_stream(self.v, None)

    def rhs(self, Q, out=None):
        out = self.empty() if out is None else out
        self._s()
        dg_varp_rhs(self.v, Q, out)
        return out

    def step(self, Q, res, dt, nsteps=1):
        self._s()
        dg_varp_rk_steps(self.v, Q, res, dt, nsteps)

    def set_timing(self, on):
        dg_varp_set_timing(self.v, on)

    def timing_read(self):
        return dg_varp_timing_read(self.v)


# ---- convenience -----------------------------------------------------------
class Solver:
    """One periodic mesh on one GPU: owns the context and a torch-allocated
    workspace, and enqueues every call on the current torch stream."""

    def __init__(self, n, p, L=(1.0, 1.0, 1.0), gamma=1.4, precision=DG_FP64, device=None, mu=0.0, prandtl=0.72,
                 volume_form=DG_VOLUME_STANDARD):
        import torch
        if isinstance(n, int):
            n = (n, n, n)
        self.n = tuple(int(v) for v in n)
        self.p = int(p)
        self.N = self.p + 1
        self.L = tuple(float(v) for v in L)
        self.gamma = float(gamma)
        self.device = torch.device(device or "cuda")
        self.ctx = dg_create(*self.n, self.p, self.gamma)
        dg_set_domain(self.ctx, *self.L)
        dg_set_precision(self.ctx, precision)
        dg_set_volume_form(self.ctx, volume_form)
        self.mu, self.prandtl = float(mu), float(prandtl)
        dg_set_viscosity(self.ctx, self.mu, self.prandtl)
        self.workspace = None
        self._workspace()

    def _workspace(self):
        """(Re)allocate the workspace the current settings need."""
        import torch
        nbytes = dg_workspace_bytes(self.ctx)
        if self.workspace is not None and self.workspace.numel() >= nbytes + 256:
            return
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        addr = self.workspace.data_ptr()
        aligned = (addr + 255) & ~255
        _check(_lib.dg_set_workspace(self.ctx, aligned, nbytes))

    def set_viscosity(self, mu, prandtl=0.72):
        """Navier-Stokes terms with dynamic viscosity mu (0: Euler)."""
        self.mu, self.prandtl = float(mu), float(prandtl)
        dg_set_viscosity(self.ctx, self.mu, self.prandtl)
        self._workspace()

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        # at interpreter exit the module's functions may already be gone
        if ctx and dg_destroy is not None:
            dg_destroy(ctx)
            self.ctx = None

    @property
    def shape(self):
        nx, ny, nz = self.n
        return (5, nz, ny, nx, self.N, self.N, self.N)

    @property
    def num_dof(self):
        return dg_num_dof(self.ctx)

    def set_precision(self, mode):
        dg_set_precision(self.ctx, mode)

    def set_option(self, key, value):
        dg_set_option(self.ctx, key, value)

    def get_option(self, key):
        return dg_get_option(self.ctx, key)

    def options(self):
        """All tuning options by name."""
        return {name: dg_get_option(self.ctx, k) for k, name in OPTION_NAMES.items()}

    def _s(self):
        dg_set_stream(self.ctx, None)

    def empty(self):
        import torch
        return torch.empty(self.shape, dtype=torch.float64, device=self.device)

    def rhs(self, Q, out=None):
        out = self.empty() if out is None else out
        self._s()
        dg_rhs(self.ctx, Q, out)
        return out

    def rk_stage(self, s, Q, res, dt):
        self._s()
        dg_rk_stage(self.ctx, s, Q, res, dt)

    def step(self, Q, res, dt, nsteps=1, graph=False):
        """nsteps LSERK45 steps in place; graph=True replays captured
        steps (dg_rk_graph_steps), bitwise the same result."""
        self._s()
        if graph:
            dg_rk_graph_steps(self.ctx, Q, res, dt, nsteps)
        else:
            dg_rk_steps(self.ctx, Q, res, dt, nsteps)

    def rhs_vjp(self, Q, gR, out=None):
        out = self.empty() if out is None else out
        self._s()
        dg_rhs_vjp(self.ctx, Q, gR, out)
        return out

    def integrals(self, Q):
        self._s()
        return dg_integrals(self.ctx, Q)

    def max_wavespeed(self, Q):
        self._s()
        return dg_max_wavespeed(self.ctx, Q)

    def dt_cfl(self, Q, cfl):
        """dt = CFL / ((2p+1) max_d-summed wave rate), computed on the GPU
        (the inviscid limit; with viscosity the caller adds any viscous
        limit)."""
        return cfl / ((2 * self.p + 1) * self.max_wavespeed(Q))

    def check_state(self, Q):
        self._s()
        return dg_check_state(self.ctx, Q)


# ---- differentiation -------------------------------------------------------
class RHS(torch.autograd.Function):
    """R = dQ/dt as an autograd function: forward dg_rhs, backward dg_rhs_vjp
    (the hand-written adjoint kernel)."""

    @staticmethod
    def forward(ctx, Q, solver):
        R = solver.rhs(Q.detach().contiguous())
        ctx.save_for_backward(Q)
        ctx.solver = solver
        return R

    @staticmethod
    def backward(ctx, gR):
        (Q,) = ctx.saved_tensors
        gQ = ctx.solver.rhs_vjp(Q.detach().contiguous(), gR.contiguous())
        return gQ, None


def rk_gradient(solver, Q0, dt, nsteps, objective_grad, every=8):
    """Gradient of an objective J(Q_nsteps) with respect to Q0 through
    ``nsteps`` LSERK45 steps, with Q checkpointed every ``every`` steps.

    objective_grad(Q) must return dJ/dQ at the final state.  Forward: one
    pass storing Q at every ``every``-th step.  Reverse, segment by segment:
    recompute the 25..40 stage inputs of the segment from its checkpoint
    (dg_rk_stage, bitwise equal to the forward pass), then run the stages
    backwards through dg_rk_stage_vjp.  Returns (J-gradient, final state)."""
    ckpts = []
    Q = Q0.detach().clone()
    res = torch.zeros_like(Q)
    for n in range(nsteps):
        if n % every == 0:
            ckpts.append(Q.clone())
        solver.step(Q, res, dt)
    Qfinal = Q
    gQ = objective_grad(Qfinal).contiguous().clone()
    gres = torch.zeros_like(gQ)
    solver._s()
    for seg in reversed(range(len(ckpts))):
        n0 = seg * every
        n1 = min(n0 + every, nsteps)
        Q = ckpts[seg].clone()
        res = torch.zeros_like(Q)
        inputs = []
        for n in range(n0, n1):
            for s in range(5):
                inputs.append((s, Q.clone()))
                solver.rk_stage(s, Q, res, dt)
        for s, Qs in reversed(inputs):
            dg_rk_stage_vjp(solver.ctx, s, Qs, gQ, gres, dt)
    return gQ, Qfinal


def kinetic_energy_grad(solver):
    """d/dQ of the integrated kinetic energy (dg_integrals' last value),
    computed by the library (dg_kinetic_energy_grad), as a function of Q."""

    def grad(Q):
        g = torch.empty_like(Q)
        solver._s()
        dg_kinetic_energy_grad(solver.ctx, Q, g)
        return g
    return grad
