"""ctypes binding of libpsatd.so (the C ABI in include/psatd.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  PyTorch supplies device memory and the current HIP stream.  If the
library has not been built, importing this module raises -- there is no
fallback path.
"""

from __future__ import annotations

import ctypes
import os
from typing import Sequence

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpsatd.so")

PSATD_OK = 0
PSATD_EINVAL = -1
PSATD_ENOMEM = -2
PSATD_EHIP = -3
PSATD_EUNSUPPORTED = -4
PSATD_ESTATE = -5
PSATD_FP32 = 0
PSATD_FP64 = 1
PSATD_FLAG_STAGGERED = 1
PSATD_FLAG_NO_WORKSPACE = 2

Q_BOX_X, Q_BOX_Y, Q_BOX_Z, Q_PRECISION, Q_WORKSPACE_BYTES, Q_SPECTRUM_POINTS, Q_Z_COLUMNS, Q_TWO_STAGE = range(8)


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("ngx", ctypes.c_int), ("ngy", ctypes.c_int), ("ngz", ctypes.c_int),
        ("order", ctypes.c_int),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("dt", ctypes.c_double), ("c", ctypes.c_double), ("eps0", ctypes.c_double),
        ("precision", ctypes.c_int), ("flags", ctypes.c_int),
    ]


class PicDesc(ctypes.Structure):
    _fields_ = [
        ("gx", ctypes.c_int), ("gy", ctypes.c_int), ("gz", ctypes.c_int),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("dt", ctypes.c_double), ("c", ctypes.c_double), ("q", ctypes.c_double), ("q_over_m", ctypes.c_double),
        ("max_particles", ctypes.c_int), ("tile", ctypes.c_int), ("precision", ctypes.c_int), ("flags", ctypes.c_int),
        ("shape", ctypes.c_int),
    ]


class PsatdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"psatd error {code}: {msg}")
        self.code = code


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """dlopen libpsatd.so and declare the C signatures (no GPU needed).

    torch is imported first: it carries its own HIP runtime under the same
    soname as the system one, and the library must bind to the runtime that
    owns torch's device memory and streams (two runtimes in one process do not
    share allocations or contexts).
    """
    import torch  # noqa: F401  (load order: torch's HIP runtime first)

    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1812_07357_amd.build_lib`")
    lib = ctypes.CDLL(path)
    vp, ip, cint = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int
    vpp = ctypes.POINTER(ctypes.c_void_p)
    lib.psatd_plan_create.restype = vp
    lib.psatd_plan_create.argtypes = [cint, cint, cint, cint, cint, ctypes.c_double, ctypes.c_double]
    lib.psatd_plan_create_ex.restype = cint
    lib.psatd_plan_create_ex.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(vp)]
    lib.psatd_plan_destroy.restype = None
    lib.psatd_plan_destroy.argtypes = [vp]
    lib.psatd_push.restype = cint
    lib.psatd_push.argtypes = [vp, vpp, vpp, vpp, vp, vp, vp]
    lib.guard_fill.restype = cint
    lib.guard_fill.argtypes = [vp, vpp, vpp, cint, ip, ip, vp]
    lib.guard_merge.restype = cint
    lib.guard_merge.argtypes = [vp, vpp, vpp, cint, ip, ip, cint, vp]
    lib.psatd_step_g1.restype = cint
    lib.psatd_step_g1.argtypes = [vp, vpp, ip, ip, vp]
    lib.psatd_step_g1_noalloc.restype = cint
    lib.psatd_step_g1_noalloc.argtypes = [vp, vpp, ip, ip, vp]
    lib.psatd_plan_query.restype = cint
    lib.psatd_plan_query.argtypes = [vp, cint, ctypes.POINTER(ctypes.c_longlong)]
    lib.psatd_plan_tables.restype = cint
    lib.psatd_plan_tables.argtypes = [vp, vp, vp]
    lib.psatd_plan_set_timing.restype = cint
    lib.psatd_plan_set_timing.argtypes = [vp, cint]
    lib.psatd_plan_pass_times.restype = cint
    lib.psatd_plan_pass_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)]
    lib.psatd_plan_autotune.restype = cint
    lib.psatd_plan_autotune.argtypes = [vp, ctypes.c_char_p, vp]
    lib.psatd_plan_schedule.restype = cint
    lib.psatd_plan_schedule.argtypes = [vp, cint, ip, cint, ip]
    lib.psatd_batch_autotune.restype = cint
    lib.psatd_batch_autotune.argtypes = [vp, ctypes.c_char_p, vp]
    lib.psatd_batch_create.restype = cint
    lib.psatd_batch_create.argtypes = [cint, ctypes.POINTER(PlanDesc), ip, ip, ctypes.POINTER(vp)]
    lib.psatd_batch_step.restype = cint
    lib.psatd_batch_step.argtypes = [vp, vpp, vp]
    lib.psatd_batch_run.restype = cint
    lib.psatd_batch_run.argtypes = [vp, vpp, cint, vp]
    lib.psatd_batch_destroy.restype = None
    lib.psatd_batch_destroy.argtypes = [vp]
    lib.psatd_batch_query.restype = cint
    lib.psatd_batch_query.argtypes = [vp, cint, ctypes.POINTER(ctypes.c_longlong)]
    fp = ctypes.POINTER(ctypes.c_float)
    cf = ctypes.c_float
    lib.psatd_mlp_create.restype = cint
    lib.psatd_mlp_create.argtypes = [fp, fp, fp, cf, cf, cint, ctypes.POINTER(vp)]
    lib.psatd_mlp_set.restype = cint
    lib.psatd_mlp_set.argtypes = [vp, fp]
    lib.psatd_mlp_get.restype = cint
    lib.psatd_mlp_get.argtypes = [vp, fp, ctypes.POINTER(ctypes.c_ushort)]
    lib.psatd_mlp_predict.restype = cint
    lib.psatd_mlp_predict.argtypes = [vp, vp, cint, vp, vp]
    lib.psatd_mlp_grad.restype = cint
    lib.psatd_mlp_grad.argtypes = [vp, vp, vp, cint, vp, cint, vp, vp, vp]
    lib.psatd_mlp_adam.restype = cint
    lib.psatd_mlp_adam.argtypes = [vp, cf, cf, cf, cf, vp]
    lib.psatd_mlp_train.restype = cint
    lib.psatd_mlp_train.argtypes = [vp, vp, vp, cint, vp, cint, cint, cf, cf, cf, cf, vp, vp]
    lib.psatd_mlp_destroy.restype = None
    lib.psatd_mlp_destroy.argtypes = [vp]
    lib.psatd_default_schedule.restype = cint
    lib.psatd_default_schedule.argtypes = [cint, ip, cint, ip]
    lib.psatd_set_device_budget.restype = cint
    lib.psatd_set_device_budget.argtypes = [ctypes.c_longlong]
    lib.psatd_device_bytes_in_use.restype = ctypes.c_longlong
    lib.psatd_device_bytes_in_use.argtypes = []
    lib.psatd_tune_cache_load.restype = cint
    lib.psatd_tune_cache_load.argtypes = [ctypes.c_char_p, ip, ip]
    lib.psatd_pml_set.argtypes = [vp, ip, ctypes.c_double, ctypes.c_double]
    lib.psatd_pml_set.restype = cint
    lib.psatd_pml_step.argtypes = [vp, vpp, vpp, vp]
    lib.psatd_pml_step.restype = cint
    lib.psatd_pic_create.argtypes = [ctypes.POINTER(PicDesc), ctypes.POINTER(vp)]
    lib.psatd_pic_create.restype = cint
    lib.psatd_pic_destroy.argtypes = [vp]
    lib.psatd_pic_destroy.restype = None
    lib.psatd_pic_push.argtypes = [vp, vpp, vpp, vpp, vpp, cint, vp]
    lib.psatd_pic_push.restype = cint
    lib.psatd_pic_deposit.argtypes = [vp, vpp, vpp, vpp, vpp, cint, vp]
    lib.psatd_pic_deposit.restype = cint
    lib.psatd_last_error.restype = ctypes.c_char_p
    lib.psatd_last_error.argtypes = []
    return lib


_lib = load_library()


def _check(rc: int):
    if rc != PSATD_OK:
        raise PsatdError(rc, _lib.psatd_last_error().decode())


def _ptrs(tensors) -> ctypes.Array:
    arr = (ctypes.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = t.data_ptr()
    return arr


def _ints(v) -> ctypes.Array:
    return (ctypes.c_int * 3)(*[int(x) for x in v])


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _triple(v):
    return (v, v, v) if isinstance(v, (int, float)) else tuple(v)


class Plan:
    """One PSATD plan: a guard-padded box of the global grid (one FFT group).

    Sizes are interior cells (x, y, z); ``nguard`` a scalar or per-axis
    triple; ``order`` 0 for infinite order, else even >= 2; ``dx`` scalar or
    triple; ``precision`` "fp32" or "fp64"; ``staggered`` for the staggered
    (Yee) grid; ``flags`` further PSATD_FLAG_* bits.
    """

    def __init__(self, nx, ny, nz, nguard=0, order=0, dx=1.0, dt=0.5, c=1.0, eps0=1.0, precision="fp32",
                 flags=0, staggered=False):
        import torch

        g = _triple(nguard)
        d = _triple(dx)
        flags = int(flags) | (PSATD_FLAG_STAGGERED if staggered else 0)
        desc = PlanDesc(int(nx), int(ny), int(nz), int(g[0]), int(g[1]), int(g[2]), int(order),
                        float(d[0]), float(d[1]), float(d[2]), float(dt), float(c), float(eps0),
                        PSATD_FP64 if precision == "fp64" else PSATD_FP32, flags)
        h = ctypes.c_void_p()
        _check(_lib.psatd_plan_create_ex(ctypes.byref(desc), ctypes.byref(h)))
        self._h = h
        self.interior = (int(nx), int(ny), int(nz))
        self.nguard = tuple(int(v) for v in g)
        self.order = int(order)
        self.dx = tuple(float(v) for v in d)
        self.dt = float(dt)
        self.c = float(c)
        self.eps0 = float(eps0)
        self.precision = "fp64" if precision == "fp64" else "fp32"
        self.staggered = bool(flags & PSATD_FLAG_STAGGERED)
        self.dtype = torch.float64 if self.precision == "fp64" else torch.float32
        self.box = (self.query(Q_BOX_X), self.query(Q_BOX_Y), self.query(Q_BOX_Z))

    # -- properties -------------------------------------------------------------
    @property
    def box_shape(self):
        """Torch shape (NZ, NY, NX) of a box array."""
        return (self.box[2], self.box[1], self.box[0])

    def query(self, what: int) -> int:
        v = ctypes.c_longlong()
        _check(_lib.psatd_plan_query(self._h, what, ctypes.byref(v)))
        return int(v.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.psatd_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- checks -------------------------------------------------------------------
    def _check_fields(self, tensors, shape, name):
        for t in tensors:
            if not t.is_cuda:
                raise ValueError(f"{name}: tensors must be on the GPU")
            if t.dtype != self.dtype:
                raise ValueError(f"{name}: dtype {t.dtype} does not match the plan ({self.dtype})")
            if not t.is_contiguous():
                raise ValueError(f"{name}: tensors must be contiguous")
            if tuple(t.shape) != tuple(shape):
                raise ValueError(f"{name}: shape {tuple(t.shape)} != {tuple(shape)}")

    @staticmethod
    def _split(fields, n):
        if hasattr(fields, "dim") and fields.dim() == 4:
            if fields.shape[0] != n:
                raise ValueError(f"expected {n} fields, got {fields.shape[0]}")
            return [fields[i] for i in range(n)]
        if len(fields) != n:
            raise ValueError(f"expected {n} fields, got {len(fields)}")
        return list(fields)

    # -- entry points -----------------------------------------------------------------
    def push(self, E: Sequence, B: Sequence, J: Sequence, rho_old, rho_new, stream=None):
        """psatd_push: advance box arrays E, B (3 each, in place) by one step."""
        allf = list(E) + list(B) + list(J) + [rho_old, rho_new]
        self._check_fields(allf, self.box_shape, "push")
        _check(_lib.psatd_push(self._h, _ptrs(E), _ptrs(B), _ptrs(J), ctypes.c_void_p(rho_old.data_ptr()),
                               ctypes.c_void_p(rho_new.data_ptr()), _stream(stream)))

    def push_fields(self, fields, stream=None):
        """push() on an (11, NZ, NY, NX) tensor (or a list of 11) in slot order."""
        f = self._split(fields, 11)
        self.push(f[0:3], f[3:6], f[6:9], f[9], f[10], stream)

    def step_g1(self, g1, origin, stream=None):
        """psatd_step_g1: fused fill + step + merge on the 11 global arrays (E, B updated in place)."""
        f = self._split(g1, 11)
        gshape = tuple(f[0].shape)
        self._check_fields(f, gshape, "step_g1")
        gdims = (gshape[2], gshape[1], gshape[0])
        _check(_lib.psatd_step_g1(self._h, _ptrs(f), _ints(origin), _ints(gdims), _stream(stream)))

    def step_g1_noalloc(self, g1, origin, stream=None):
        """psatd_step_g1_noalloc: the fused step with its workspace in the library's static scratch."""
        f = self._split(g1, 11)
        gshape = tuple(f[0].shape)
        self._check_fields(f, gshape, "step_g1_noalloc")
        gdims = (gshape[2], gshape[1], gshape[0])
        _check(_lib.psatd_step_g1_noalloc(self._h, _ptrs(f), _ints(origin), _ints(gdims), _stream(stream)))

    def pml_set(self, widths, sigma_max, power=2.0):
        """psatd_pml_set: absorbing layers of ``widths`` (x, y, z) cells at both ends of each axis."""
        _check(_lib.psatd_pml_set(self._h, _ints(widths), float(sigma_max), float(power)))

    def pml_step(self, parts, sources, stream=None):
        """psatd_pml_step: one step of the 12 split parts (in place) with the 5 sources
        (Jx Jy Jz rho_old rho_new), all box arrays."""
        p = self._split(parts, 12)
        src = self._split(sources, 5)
        self._check_fields(p + src, self.box_shape, "pml_step")
        _check(_lib.psatd_pml_step(self._h, _ptrs(p), _ptrs(src), _stream(stream)))

    def guard_fill(self, g1, box, origin, stream=None):
        """guard_fill: gather box arrays (interior + guards) from the periodic global arrays."""
        g = list(g1)
        b = list(box)
        if len(g) != len(b) or not g:
            raise ValueError("guard_fill: g1 and box must hold the same number of arrays")
        gshape = tuple(g[0].shape)
        self._check_fields(g, gshape, "guard_fill g1")
        self._check_fields(b, self.box_shape, "guard_fill box")
        gdims = (gshape[2], gshape[1], gshape[0])
        _check(_lib.guard_fill(self._h, _ptrs(g), _ptrs(b), len(g), _ints(origin), _ints(gdims), _stream(stream)))

    def guard_merge(self, box, g1, origin, mode=0, stream=None):
        """guard_merge: copy (mode 0) or add (mode 1) box arrays back into the global arrays."""
        g = list(g1)
        b = list(box)
        if len(g) != len(b) or not g:
            raise ValueError("guard_merge: g1 and box must hold the same number of arrays")
        gshape = tuple(g[0].shape)
        self._check_fields(g, gshape, "guard_merge g1")
        self._check_fields(b, self.box_shape, "guard_merge box")
        gdims = (gshape[2], gshape[1], gshape[0])
        _check(_lib.guard_merge(self._h, _ptrs(b), _ptrs(g), len(g), _ints(origin), _ints(gdims), int(mode),
                                _stream(stream)))

    def autotune(self, cache_path=None, stream=None):
        """Time candidate radix orders / tile sizes per axis and keep the fastest (JSON cache optional)."""
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(_lib.psatd_plan_autotune(self._h, path, _stream(stream)))

    def schedule(self, axis: int):
        """(radix sequence, tile parameter) currently used along axis 0 (x), 1 (y) or 2 (z)."""
        buf = (ctypes.c_int * 16)()
        tile = ctypes.c_int()
        n = _lib.psatd_plan_schedule(self._h, int(axis), buf, 16, ctypes.byref(tile))
        if n < 0:
            _check(n)
        return list(buf[:n]), int(tile.value)

    PASS_NAMES = ("x_fwd_fill", "y_fwd", "z_push", "y_inv", "x_inv_merge")

    def set_timing(self, enable: bool):
        """Record HIP events around each pass of every following step."""
        _check(_lib.psatd_plan_set_timing(self._h, 1 if enable else 0))

    def pass_times(self):
        """Mean milliseconds per pass since timing was enabled (waits for the last step)."""
        ms = (ctypes.c_double * 5)()
        n = ctypes.c_longlong()
        _check(_lib.psatd_plan_pass_times(self._h, ms, ctypes.byref(n)))
        return dict(zip(self.PASS_NAMES, list(ms))), int(n.value)

    def tables(self, stream=None):
        """Coefficient tables (5, NXH, NY, NZ) and 1D modified k (kx, ky, kz) at working precision."""
        import torch

        npts = self.query(Q_SPECTRUM_POINTS)
        NX, NY, NZ = self.box
        nxh = NX // 2 + 1
        buf = torch.empty(5 * npts + nxh + NY + NZ, dtype=self.dtype, device="cuda")
        _check(_lib.psatd_plan_tables(self._h, ctypes.c_void_p(buf.data_ptr()), _stream(stream)))
        coef = buf[: 5 * npts].view(5, nxh, NY, NZ)
        k = buf[5 * npts:]
        return coef, k[:nxh], k[nxh:nxh + NY], k[nxh + NY:]


QB_BOXES, QB_TILES, QB_BOX_CELLS, QB_INTERIOR_CELLS, QB_WORKSPACE_BYTES = range(5)


class Batch:
    """Many boxes of one periodic global grid, advanced together (psatd_batch_*).

    ``boxes``: iterable of dicts with ``origin`` (x, y, z), ``interior``
    (nx, ny, nz), ``nguard`` (scalar or triple), ``order`` and optionally
    ``staggered`` (Yee grid, PSATD_FLAG_STAGGERED); ``gdims`` =
    (GX, GY, GZ).  Each pass of a step is one persistent launch per class of boxes
    (same block size, similar LDS size);
    ``run`` replays ``nsteps`` steps from a captured hipGraph.
    """

    def __init__(self, boxes, gdims, dx=1.0, dt=0.5, c=1.0, eps0=1.0, precision="fp32"):
        import torch

        boxes = list(boxes)
        d = _triple(dx)
        descs = (PlanDesc * len(boxes))()
        origins = (ctypes.c_int * (3 * len(boxes)))()
        for i, b in enumerate(boxes):
            g = _triple(b["nguard"])
            n = b["interior"]
            descs[i] = PlanDesc(int(n[0]), int(n[1]), int(n[2]), int(g[0]), int(g[1]), int(g[2]), int(b["order"]),
                                float(d[0]), float(d[1]), float(d[2]), float(dt), float(c), float(eps0),
                                PSATD_FP64 if precision == "fp64" else PSATD_FP32,
                                PSATD_FLAG_STAGGERED if b.get("staggered", False) else 0)
            for a in range(3):
                origins[3 * i + a] = int(b["origin"][a])
        h = ctypes.c_void_p()
        _check(_lib.psatd_batch_create(len(boxes), descs, origins, _ints(gdims), ctypes.byref(h)))
        self._h = h
        self.boxes = boxes
        self.gdims = tuple(int(v) for v in gdims)
        self.precision = "fp64" if precision == "fp64" else "fp32"
        self.dtype = torch.float64 if self.precision == "fp64" else torch.float32

    def query(self, what: int) -> int:
        v = ctypes.c_longlong()
        _check(_lib.psatd_batch_query(self._h, what, ctypes.byref(v)))
        return int(v.value)

    def _fields(self, g1):
        f = Plan._split(g1, 11)
        shape = (self.gdims[2], self.gdims[1], self.gdims[0])
        for t in f:
            if not t.is_cuda or t.dtype != self.dtype or not t.is_contiguous() or tuple(t.shape) != shape:
                raise ValueError(f"g1 arrays must be contiguous {self.dtype} GPU tensors of shape {shape}")
        return f

    def autotune(self, cache_path=None, stream=None):
        """Autotune every box plan (psatd_batch_autotune)."""
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(_lib.psatd_batch_autotune(self._h, path, _stream(stream)))

    def step(self, g1, stream=None):
        """One step of every box (eager launches)."""
        _check(_lib.psatd_batch_step(self._h, _ptrs(self._fields(g1)), _stream(stream)))

    def run(self, g1, nsteps: int, stream=None):
        """``nsteps`` steps replayed from a hipGraph (captured on first use)."""
        _check(_lib.psatd_batch_run(self._h, _ptrs(self._fields(g1)), int(nsteps), _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.psatd_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pic:
    """Particle side of the PIC cycle on the global grid G1 (psatd_pic_*).

    ``gdims`` = (GX, GY, GZ); ``tile`` the D1 tile edge; ``shape`` the degree
    of the particle shape (1 cloud in cell, 2 triangular-shaped cloud, 3 cubic
    B-spline) used by both gather and deposit; particles are (3, n) tensors of
    positions ``x`` and momenta per mass ``u`` (x, y, z rows), of the object's
    precision, on the GPU.
    """

    def __init__(self, gdims, dx=1.0, dt=0.5, c=1.0, q=1.0, q_over_m=1.0, max_particles=1 << 20, tile=8,
                 precision="fp32", staggered=False, shape=1):
        import torch

        d = _triple(dx)
        desc = PicDesc(int(gdims[0]), int(gdims[1]), int(gdims[2]), float(d[0]), float(d[1]), float(d[2]),
                       float(dt), float(c), float(q), float(q_over_m), int(max_particles), int(tile),
                       PSATD_FP64 if precision == "fp64" else PSATD_FP32,
                       PSATD_FLAG_STAGGERED if staggered else 0, int(shape))
        h = ctypes.c_void_p()
        _check(_lib.psatd_pic_create(ctypes.byref(desc), ctypes.byref(h)))
        self._h = h
        self.gdims = tuple(int(v) for v in gdims)
        self.max_particles = int(max_particles)
        self.shape = int(shape) if shape else 1
        self.precision = "fp64" if precision == "fp64" else "fp32"
        self.dtype = torch.float64 if self.precision == "fp64" else torch.float32

    def _parts(self, name, t, n=None):
        if not t.is_cuda or t.dtype != self.dtype or t.dim() != 2 or t.shape[0] != 3:
            raise ValueError(f"{name}: expected a (3, n) {self.dtype} GPU tensor")
        if n is not None and t.shape[1] != n:
            raise ValueError(f"{name}: expected {n} particles, got {t.shape[1]}")
        rows = [t[k] for k in range(3)]
        if not all(r.is_contiguous() for r in rows):
            raise ValueError(f"{name}: rows must be contiguous")
        return rows

    def _g1(self, g1):
        f = Plan._split(g1, 11)
        shape = (self.gdims[2], self.gdims[1], self.gdims[0])
        for t in f:
            if not t.is_cuda or t.dtype != self.dtype or not t.is_contiguous() or tuple(t.shape) != shape:
                raise ValueError(f"g1 arrays must be contiguous {self.dtype} GPU tensors of shape {shape}")
        return f

    def push(self, g1, x, u, x_old, stream=None):
        """psatd_pic_push: gather E, B at x, Boris-push u, move x (in place); x_old receives the old x."""
        n = x.shape[1]
        xs, us, xo = self._parts("x", x), self._parts("u", u, n), self._parts("x_old", x_old, n)
        _check(_lib.psatd_pic_push(self._h, _ptrs(self._g1(g1)), _ptrs(xs), _ptrs(us), _ptrs(xo), int(n),
                                   _stream(stream)))

    def deposit(self, g1, x_old, x, u, stream=None):
        """psatd_pic_deposit: J (mid-point), rho_old, rho_new into g1 slots 6..10 (overwritten)."""
        n = x.shape[1]
        xo, xs, us = self._parts("x_old", x_old, n), self._parts("x", x), self._parts("u", u, n)
        _check(_lib.psatd_pic_deposit(self._h, _ptrs(self._g1(g1)), _ptrs(xo), _ptrs(xs), _ptrs(us), int(n),
                                      _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.psatd_pic_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MLP_NPARAM = 4673


class Mlp:
    """Guard-width surrogate network (psatd_mlp_*): 6 -> 64 -> 64 -> 1, SiLU, bfloat16 weights.

    ``init``: MLP_NPARAM initial FP32 parameters (W1, b1, W2, b2, W3, b3);
    ``in_mean`` / ``in_scale``: per-feature standardisation; ``out_mean`` /
    ``out_scale``: affine map of the network output to log10 error.
    Every tensor argument is a contiguous GPU tensor (float32 features
    (n, 6) and targets (n,), int32 indices).
    """

    def __init__(self, init, in_mean, in_scale, out_mean=0.0, out_scale=1.0, max_batch=4096):
        import numpy as np

        init = np.ascontiguousarray(init, dtype=np.float32)
        if init.shape != (MLP_NPARAM,):
            raise ValueError(f"init must hold {MLP_NPARAM} values")
        mean = np.ascontiguousarray(in_mean, dtype=np.float32).reshape(6)
        scale = np.ascontiguousarray(in_scale, dtype=np.float32).reshape(6)
        fp = ctypes.POINTER(ctypes.c_float)
        h = ctypes.c_void_p()
        _check(_lib.psatd_mlp_create(init.ctypes.data_as(fp), mean.ctypes.data_as(fp), scale.ctypes.data_as(fp),
                                     float(out_mean), float(out_scale), int(max_batch), ctypes.byref(h)))
        self._h = h
        self.max_batch = int(max_batch)
        self.norm = (mean.copy(), scale.copy(), float(out_mean), float(out_scale))

    @staticmethod
    def _gpu(t, dtype, shape=None, name="tensor"):
        if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dtype} GPU tensor")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        return ctypes.c_void_p(t.data_ptr())

    def _xt(self, X, t=None):
        import torch

        if X.dim() != 2 or X.shape[1] != 6:
            raise ValueError("features must have shape (n, 6)")
        n = int(X.shape[0])
        px = self._gpu(X, torch.float32, name="features")
        pt = None if t is None else self._gpu(t, torch.float32, (n,), "targets")
        return n, px, pt

    def set_params(self, master):
        import numpy as np

        m = np.ascontiguousarray(master, dtype=np.float32)
        if m.shape != (MLP_NPARAM,):
            raise ValueError(f"parameters must hold {MLP_NPARAM} values")
        _check(_lib.psatd_mlp_set(self._h, m.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def params(self):
        """(FP32 master weights, bfloat16 copy as float32) as numpy arrays (synchronises)."""
        import numpy as np

        m = np.empty(MLP_NPARAM, dtype=np.float32)
        b = np.empty(MLP_NPARAM, dtype=np.uint16)
        _check(_lib.psatd_mlp_get(self._h, m.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                  b.ctypes.data_as(ctypes.POINTER(ctypes.c_ushort))))
        return m, (b.astype(np.uint32) << 16).view(np.float32)

    def predict(self, X, stream=None):
        import torch

        n, px, _ = self._xt(X)
        y = torch.empty(n, dtype=torch.float32, device=X.device)
        _check(_lib.psatd_mlp_predict(self._h, px, n, ctypes.c_void_p(y.data_ptr()), _stream(stream)))
        return y

    def grad(self, X, t, idx=None, batch=None, stream=None):
        """(gradient (MLP_NPARAM,), loss) of the batch as GPU tensors."""
        import torch

        n, px, pt = self._xt(X, t)
        pi = None
        if idx is not None:
            pi = self._gpu(idx, torch.int32, name="idx")
            batch = int(idx.numel()) if batch is None else int(batch)
        batch = n if batch is None else int(batch)
        g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=X.device)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        _check(_lib.psatd_mlp_grad(self._h, px, pt, n, pi, batch, ctypes.c_void_p(g.data_ptr()),
                                   ctypes.c_void_p(loss.data_ptr()), _stream(stream)))
        return g, loss

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(_lib.psatd_mlp_adam(self._h, lr, beta1, beta2, eps, _stream(stream)))

    def train(self, X, t, idx, nsteps, batch, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        """``nsteps`` Adam steps on minibatches idx[k*batch:(k+1)*batch]; returns the per-step loss (GPU)."""
        import torch

        n, px, pt = self._xt(X, t)
        pi = None
        if idx is not None:
            if idx.numel() < int(nsteps) * int(batch):
                raise ValueError("idx must hold nsteps * batch indices")
            pi = self._gpu(idx, torch.int32, name="idx")
        hist = torch.empty(max(1, int(nsteps)), dtype=torch.float32, device=X.device)
        _check(_lib.psatd_mlp_train(self._h, px, pt, n, pi, int(nsteps), int(batch), lr, beta1, beta2, eps,
                                    ctypes.c_void_p(hist.data_ptr()), _stream(stream)))
        return hist[: int(nsteps)]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.psatd_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_schedule(n: int):
    """(radices, transform length) of the build's default line schedule for an edge of n cells (host only)."""
    r = (ctypes.c_int * 16)()
    m = ctypes.c_int()
    ns = _lib.psatd_default_schedule(int(n), r, 16, ctypes.byref(m))
    _check(ns if ns < 0 else PSATD_OK)
    return [r[i] for i in range(ns)], m.value


def set_device_budget(nbytes):
    """Cap the device bytes the library's plans and batches may hold (None: no cap)."""
    _check(_lib.psatd_set_device_budget(-1 if nbytes is None else int(nbytes)))


def device_bytes_in_use() -> int:
    """Device bytes currently held by the library's plans and batches."""
    return int(_lib.psatd_device_bytes_in_use())


def tune_cache_load(path):
    """Read an autotuner cache file into the process cache (host only): (accepted, rejected) entries."""
    a, r = ctypes.c_int(), ctypes.c_int()
    _check(_lib.psatd_tune_cache_load(os.fsencode(path), ctypes.byref(a), ctypes.byref(r)))
    return int(a.value), int(r.value)
