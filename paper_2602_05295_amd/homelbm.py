"""ctypes binding of libhomelbm.so (include/homelbm.h).

Argument marshalling only: every step of the method runs in the HIP library.
Arrays may be numpy arrays (host) or torch CUDA tensors (device); torch is
used only for device memory and streams.  There is no CPU fallback: if the
library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhomelbm.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "homelbm.h")

FP32, Q16 = 0, 1
# b_rho_u / b_S bit allocations (codes of rho and u with b1 bits, of N with b2)
PACKED = {"p16_15": (2, 16, 15), "p15_14": (3, 15, 14), "p14_13": (4, 14, 13), "p13_12": (5, 13, 12),
          "p12_11": (6, 12, 11)}
FORMATS = {"fp32": FP32, "q16": Q16, **{k: v[0] for k, v in PACKED.items()}}
BITS = {Q16: (16, 16), **{v[0]: (v[1], v[2]) for v in PACKED.values()}}


def raw_planes(fmt: int) -> int:
    """Planes of the raw state: 10 floats, or ceil((4 b1 + 6 b2)/32) words."""
    if fmt == FP32:
        return 10
    b1, b2 = BITS[fmt]
    return (4 * b1 + 6 * b2 + 31) // 32


def _fmt_code(fmt):
    if isinstance(fmt, str):
        return FORMATS[fmt]
    if int(fmt) in BITS or int(fmt) == FP32:
        return int(fmt)
    raise KeyError(fmt)
DITHER_OFF, DITHER_PER_STEP, DITHER_STATIC = 0, 1, 2
OK, ERR_INVALID_ARG, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_UNSUPPORTED, ERR_UNSTABLE = range(6)
_STATUS = {0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "DEVICE", 4: "UNSUPPORTED", 5: "UNSTABLE"}


class LBMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [
        ("dither_mode", ctypes.c_int),
        ("seed", ctypes.c_uint32),
        ("inflow", ctypes.c_int),
        ("u_in", ctypes.c_float * 3),
        ("check_health", ctypes.c_int),
        ("tile_rows", ctypes.c_int),
        ("force", ctypes.c_float * 3),
        ("wall_rule", ctypes.c_int),
        ("track_forces", ctypes.c_int),
        ("pipeline", ctypes.c_int),
        ("graph_steps", ctypes.c_int),
    ]


class BatchTuning(ctypes.Structure):
    _fields_ = [
        ("block", ctypes.c_int),
        ("wg_per_cu", ctypes.c_int),
        ("workgroups", ctypes.c_int),
        ("segments", ctypes.c_int),
        ("balance", ctypes.c_double),
        ("fluid_ms", ctypes.c_double),
        ("from_cache", ctypes.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def declared_functions():
    """Names of the functions include/homelbm.h declares."""
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def lib():
    """Loads libhomelbm.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2602_05295_amd.build` "
                           "(or __graft_entry__.build()); there is no fallback")
    # One HIP runtime per process: torch ships its own libamdhip64 (soname
    # libamdhip64.so.7) and asks for it by file name.  Loaded first, it
    # satisfies this library's libamdhip64.so.7 too; loaded after this
    # library, it would be a second runtime that finds no GPU.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    P = ctypes.POINTER
    L.lbm_default_options.argtypes = [P(Options)]
    L.lbm_create.argtypes = [P(ctypes.c_int), ctypes.c_double, vp, i, P(vp)]
    L.lbm_destroy.argtypes = [vp]
    L.lbm_last_error.argtypes = [vp]
    L.lbm_last_error.restype = ctypes.c_char_p
    L.lbm_set_stream.argtypes = [vp, vp]
    L.lbm_set_options.argtypes = [vp, P(Options)]
    L.lbm_get_options.argtypes = [vp, P(Options)]
    L.lbm_set_moments.argtypes = [vp, vp, i]
    L.lbm_set_equilibrium.argtypes = [vp, vp, vp, i]
    L.lbm_step.argtypes = [vp, i]
    L.lbm_prepare.argtypes = [vp, i]
    L.lbm_step_into.argtypes = [vp, vp, vp]
    L.lbm_set_object.argtypes = [vp, i, vp, vp, vp]
    L.lbm_get_object_forces.argtypes = [vp, vp, i]
    L.lbm_profile_stages.argtypes = [vp, i, vp]
    L.lbm_get_moments.argtypes = [vp, vp, i]
    L.lbm_raw_bytes.argtypes = [vp]
    L.lbm_raw_bytes.restype = sz
    L.lbm_get_raw.argtypes = [vp, vp, sz, i]
    L.lbm_set_raw.argtypes = [vp, vp, sz, i]
    L.lbm_get_step_count.argtypes = [vp, P(ctypes.c_uint64)]
    L.lbm_set_step_count.argtypes = [vp, ctypes.c_uint64]
    L.lbm_memory_bytes.argtypes = [vp, P(sz), P(sz)]
    L.lbm_boundary_counts.argtypes = [vp, P(ctypes.c_int64), P(ctypes.c_int64)]
    L.lbm_tile_rows.argtypes = [vp, P(ctypes.c_int)]
    L.lbm_check.argtypes = [vp, P(ctypes.c_uint64)]
    L.lbm_synchronize.argtypes = [vp]
    L.lbm_profile_steps.argtypes = [vp, i, P(ctypes.c_double), P(ctypes.c_double), P(i), P(i)]
    L.lbm_debug_dither.argtypes = [i, vp, ctypes.c_uint32, ctypes.c_uint32, i, vp]
    L.lbm_set_triangles.argtypes = [vp, ctypes.c_int64, vp, vp]
    L.lbm_adjoint_step.argtypes = [vp, vp, vp, vp]
    L.lbm_adjoint_step_noalloc.argtypes = [vp, vp, vp, vp]
    L.lbm_equilibrium_vjp.argtypes = [vp, vp, vp, vp, vp, vp]
    L.lbm_fluid_plan.argtypes = [P(i), i, i, P(i)]
    # batched API
    L.lbm_batch_create.argtypes = [i, P(i), P(ctypes.c_double), P(vp), i, P(vp)]
    L.lbm_batch_destroy.argtypes = [vp]
    L.lbm_batch_last_error.argtypes = [vp]
    L.lbm_batch_last_error.restype = ctypes.c_char_p
    L.lbm_batch_set_stream.argtypes = [vp, vp]
    L.lbm_batch_set_options.argtypes = [vp, P(Options)]
    L.lbm_batch_get_options.argtypes = [vp, P(Options)]
    L.lbm_batch_info.argtypes = [vp, i, P(i), P(ctypes.c_int64), P(ctypes.c_int64)]
    L.lbm_batch_total_cells.argtypes = [vp, P(ctypes.c_int64)]
    L.lbm_batch_set_moments.argtypes = [vp, i, vp, i]
    L.lbm_batch_set_equilibrium.argtypes = [vp, i, vp, vp, i]
    L.lbm_batch_get_moments.argtypes = [vp, i, vp, i]
    L.lbm_batch_raw_bytes.argtypes = [vp, i]
    L.lbm_batch_raw_bytes.restype = sz
    L.lbm_batch_get_raw.argtypes = [vp, i, vp, sz, i]
    L.lbm_batch_set_raw.argtypes = [vp, i, vp, sz, i]
    L.lbm_batch_step.argtypes = [vp, i]
    L.lbm_batch_step_eager.argtypes = [vp, i]
    L.lbm_batch_profile_steps.argtypes = [vp, i, P(ctypes.c_double), P(ctypes.c_double)]
    L.lbm_batch_get_step_count.argtypes = [vp, P(ctypes.c_uint64)]
    L.lbm_batch_set_step_count.argtypes = [vp, ctypes.c_uint64]
    L.lbm_batch_boundary_counts.argtypes = [vp, P(ctypes.c_int64), P(ctypes.c_int64)]
    L.lbm_batch_memory_bytes.argtypes = [vp, P(sz), P(sz)]
    L.lbm_batch_check.argtypes = [vp, P(ctypes.c_uint64)]
    L.lbm_batch_synchronize.argtypes = [vp]
    L.lbm_batch_tune.argtypes = [vp, ctypes.c_char_p, P(BatchTuning)]
    L.lbm_batch_get_tuning.argtypes = [vp, P(BatchTuning)]
    L.lbm_batch_set_tuning.argtypes = [vp, i, i]
    L.lbm_batch_plan.argtypes = [i, P(i), i, i, P(i), P(ctypes.c_uint16), P(ctypes.c_uint32), P(i),
                                 P(ctypes.c_double)]
    _lib = L
    return L


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr(a, dtype, count):
    """(pointer, on_device, keepalive) for a numpy array or a torch CUDA tensor."""
    if _is_torch(a):
        if not a.is_cuda or not a.is_contiguous():
            raise ValueError("torch tensors must be contiguous CUDA tensors")
        if a.numel() != count or a.element_size() != np.dtype(dtype).itemsize:
            raise ValueError(f"tensor must hold {count} values of {np.dtype(dtype)}")
        return ctypes.c_void_p(a.data_ptr()), 1, a
    arr = np.ascontiguousarray(a, dtype=dtype)
    if arr.size != count:
        raise ValueError(f"array must hold {count} values, has {arr.size}")
    return arr.ctypes.data_as(ctypes.c_void_p), 0, arr


def debug_dither(idx, t, seed, mode):
    """Device-side dither hash words (n, 2) for host cell indices idx."""
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    out = np.zeros((idx.size, 2), dtype=np.uint32)
    st = lib().lbm_debug_dither(idx.size, idx.ctypes.data_as(ctypes.c_void_p), t, seed, mode,
                                out.ctypes.data_as(ctypes.c_void_p))
    if st != OK:
        raise LBMError(st, lib().lbm_last_error(None).decode())
    return out


def fluid_plan(dims, tile_rows=0, cus=256):
    """The fluid pass's work split (host only): dict of tile rows, tiles along
    x and y, z segments per tile, workgroups launched, planes in the tail and
    the workgroups on it."""
    d = (ctypes.c_int * 3)(*[int(v) for v in dims])
    out = (ctypes.c_int * 7)()
    st = lib().lbm_fluid_plan(d, int(tile_rows), int(cus), out)
    if st != OK:
        raise LBMError(st, lib().lbm_last_error(None).decode())
    return dict(zip(("rows", "ntx", "nty", "nseg", "nwg", "tail", "ntail"), list(out)))


class HomeLBM:
    """One HOME-LBM domain on the current HIP device."""

    def __init__(self, dims, tau, mask=None, fmt="fp32", stream=None, **options):
        L = lib()
        self.dims = tuple(int(d) for d in dims)
        self.N = int(np.prod(self.dims))
        self.fmt = _fmt_code(fmt)
        d = (ctypes.c_int * 3)(*self.dims)
        self._mask = None
        mp = None
        if mask is not None:
            self._mask = np.ascontiguousarray(mask, dtype=np.uint8)
            if self._mask.size != self.N:
                raise ValueError("mask must have nx*ny*nz entries")
            mp = self._mask.ctypes.data_as(ctypes.c_void_p)
        h = ctypes.c_void_p()
        self._h = None
        self._check(L.lbm_create(d, float(tau), mp, self.fmt, ctypes.byref(h)), None)
        self._h = h
        self.tau = float(tau)
        if stream is None:
            stream = _torch_stream()
        if stream is not None:
            self._check(L.lbm_set_stream(self._h, ctypes.c_void_p(stream)))
        if options:
            self.set_options(**options)

    # -- plumbing
    def _check(self, st, h="self"):
        if st != OK:
            handle = self._h if h == "self" else h
            msg = lib().lbm_last_error(handle)
            raise LBMError(st, msg.decode() if msg else "")
        return st

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- options
    def options(self) -> Options:
        o = Options()
        self._check(lib().lbm_get_options(self._h, ctypes.byref(o)))
        return o

    def set_options(self, dither_mode=None, seed=None, inflow=None, u_in=None, check_health=None, tile_rows=None,
                    force=None, wall_rule=None, track_forces=None, pipeline=None, graph_steps=None):
        o = self.options()
        if dither_mode is not None:
            o.dither_mode = int(dither_mode)
        if seed is not None:
            o.seed = int(seed) & 0xFFFFFFFF
        if inflow is not None:
            o.inflow = int(bool(inflow))
        if u_in is not None:
            o.u_in = (ctypes.c_float * 3)(*[float(v) for v in u_in])
        if check_health is not None:
            o.check_health = int(bool(check_health))
        if tile_rows is not None:
            o.tile_rows = int(tile_rows)
        if force is not None:
            o.force = (ctypes.c_float * 3)(*[float(v) for v in force])
        if wall_rule is not None:
            o.wall_rule = int(wall_rule)
        if track_forces is not None:
            o.track_forces = int(bool(track_forces))
        if pipeline is not None:
            o.pipeline = int(pipeline)
        if graph_steps is not None:
            o.graph_steps = int(graph_steps)
        self._check(lib().lbm_set_options(self._h, ctypes.byref(o)))

    def set_object(self, oid, center=(0.0, 0.0, 0.0), velocity=(0.0, 0.0, 0.0), omega=(0.0, 0.0, 0.0)):
        """Wall motion of solid object oid (its mask value) and its torque center."""
        f3 = lambda v: (ctypes.c_float * 3)(*[float(x) for x in v])
        self._check(lib().lbm_set_object(self._h, int(oid), f3(center), f3(velocity), f3(omega)))

    def set_triangles(self, tris, obj):
        """Obstacle meshes of wall rule 2: tris (T, 9) float32 vertices, obj (T,)
        uint8 object ids (host arrays)."""
        t = np.ascontiguousarray(tris, dtype=np.float32).reshape(-1, 9)
        o = np.ascontiguousarray(obj, dtype=np.uint8).reshape(-1)
        if o.size != t.shape[0]:
            raise ValueError("one object id per triangle")
        self._check(lib().lbm_set_triangles(self._h, int(t.shape[0]), t.ctypes.data_as(ctypes.c_void_p),
                                            o.ctypes.data_as(ctypes.c_void_p)))

    def profile_stages(self, n):
        """Runs n steps; summed device ms of the fluid / stream pass, the boundary
        pass / link corrections, and the requantize pass (pipeline 1)."""
        ms = np.zeros(3, np.float64)
        self._check(lib().lbm_profile_stages(self._h, int(n), ms.ctypes.data_as(ctypes.c_void_p)))
        return {"fluid_ms": ms[0], "boundary_ms": ms[1], "requantize_ms": ms[2], "steps": int(n)}

    def object_forces(self, reset=False):
        """(256, 6) sums of force and torque per object id since the last reset."""
        out = np.zeros((256, 6), np.float64)
        self._check(lib().lbm_get_object_forces(self._h, out.ctypes.data_as(ctypes.c_void_p), int(bool(reset))))
        return out

    def set_stream(self, stream):
        self._check(lib().lbm_set_stream(self._h, ctypes.c_void_p(stream or 0)))

    # -- state
    def set_moments(self, m):
        p, dev, keep = _ptr(m, np.float32, 10 * self.N)
        self._check(lib().lbm_set_moments(self._h, p, dev))

    def set_equilibrium(self, rho, u):
        p1, d1, k1 = _ptr(rho, np.float32, self.N)
        p2, d2, k2 = _ptr(u, np.float32, 3 * self.N)
        if d1 != d2:
            raise ValueError("rho and u must both be host arrays or both device tensors")
        self._check(lib().lbm_set_equilibrium(self._h, p1, p2, d1))

    def get_moments(self, out=None):
        """(10, nz, ny, nx) float32 numpy array, or fills a torch CUDA tensor."""
        if out is None:
            out = np.empty((10,) + self.dims[::-1], dtype=np.float32)
        p, dev, keep = _ptr(out, np.float32, 10 * self.N)
        self._check(lib().lbm_get_moments(self._h, p, dev))
        return out

    def raw_bytes(self):
        return int(lib().lbm_raw_bytes(self._h))

    def get_raw(self, out=None):
        """Raw state: FP32 (10, nz, ny, nx) float32, integer formats (W, nz, ny, nx) uint32."""
        shape = (raw_planes(self.fmt),) + self.dims[::-1]
        dt = np.float32 if self.fmt == FP32 else np.uint32
        if out is None:
            out = np.empty(shape, dtype=dt)
        p, dev, keep = _ptr(out, dt, int(np.prod(shape)))
        self._check(lib().lbm_get_raw(self._h, p, self.raw_bytes(), dev))
        return out

    def set_raw(self, raw):
        dt = np.float32 if self.fmt == FP32 else np.uint32
        n = raw_planes(self.fmt) * self.N
        p, dev, keep = _ptr(raw, dt, n)
        self._check(lib().lbm_set_raw(self._h, p, self.raw_bytes(), dev))

    # -- stepping
    def step(self, n=1):
        self._check(lib().lbm_step(self._h, int(n)))

    def prepare(self, n):
        """Capture ahead of time what step(n) replays (no step is taken)."""
        self._check(lib().lbm_prepare(self._h, int(n)))

    def step_into(self, raw_in, raw_out):
        """One step from the raw state raw_in to raw_out (device tensors in the
        get_raw layout); the context's own state is left as it is."""
        dt = np.float32 if self.fmt == FP32 else np.uint32
        n = raw_planes(self.fmt) * self.N
        p1, d1, k1 = _ptr(raw_in, dt, n)
        p2, d2, k2 = _ptr(raw_out, dt, n)
        if not (d1 and d2):
            raise ValueError("step_into takes device tensors")
        self._check(lib().lbm_step_into(self._h, p1, p2))

    def synchronize(self):
        self._check(lib().lbm_synchronize(self._h))

    @property
    def step_count(self):
        t = ctypes.c_uint64()
        self._check(lib().lbm_get_step_count(self._h, ctypes.byref(t)))
        return t.value

    @step_count.setter
    def step_count(self, t):
        self._check(lib().lbm_set_step_count(self._h, int(t)))

    def memory_bytes(self):
        s, t = ctypes.c_size_t(), ctypes.c_size_t()
        self._check(lib().lbm_memory_bytes(self._h, ctypes.byref(s), ctypes.byref(t)))
        return s.value, t.value

    def boundary_counts(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().lbm_boundary_counts(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    @property
    def tile_rows(self):
        """The fluid pass's tile height in use (0 before the context has timed them)."""
        r = ctypes.c_int()
        self._check(lib().lbm_tile_rows(self._h, ctypes.byref(r)))
        return r.value

    def check(self):
        bad = ctypes.c_uint64()
        st = lib().lbm_check(self._h, ctypes.byref(bad))
        if st not in (OK, ERR_UNSTABLE):
            self._check(st)
        return bad.value

    # -- adjoint (FP32 contexts; torch CUDA tensors)
    def adjoint_step(self, m_t, lam_next, lam_prev):
        """lam_prev <- J(m_t)^T lam_next; m_t is a raw FP32 state (get_raw layout)."""
        n = 10 * self.N
        p1, d1, k1 = _ptr(m_t, np.float32, n)
        p2, d2, k2 = _ptr(lam_next, np.float32, n)
        p3, d3, k3 = _ptr(lam_prev, np.float32, n)
        if not (d1 and d2 and d3):
            raise ValueError("adjoint_step takes device tensors")
        self._check(lib().lbm_adjoint_step(self._h, p1, p2, p3))

    def equilibrium_vjp(self, rho, u, lam, grad_u, grad_rho=None):
        p1, d1, k1 = _ptr(rho, np.float32, self.N)
        p2, d2, k2 = _ptr(u, np.float32, 3 * self.N)
        p3, d3, k3 = _ptr(lam, np.float32, 10 * self.N)
        p4, d4, k4 = _ptr(grad_u, np.float32, 3 * self.N)
        p5 = None
        if grad_rho is not None:
            p5, d5, k5 = _ptr(grad_rho, np.float32, self.N)
        if not (d1 and d2 and d3 and d4):
            raise ValueError("equilibrium_vjp takes device tensors")
        self._check(lib().lbm_equilibrium_vjp(self._h, p1, p2, p3, p5, p4))

    def profile_steps(self, n):
        """Runs n steps with per-kernel HIP events: dict of summed ms and launch counts."""
        f, b = ctypes.c_double(), ctypes.c_double()
        nf, nb = ctypes.c_int(), ctypes.c_int()
        self._check(lib().lbm_profile_steps(self._h, int(n), ctypes.byref(f), ctypes.byref(b), ctypes.byref(nf),
                                            ctypes.byref(nb)))
        return {"fluid_ms": f.value, "boundary_ms": b.value, "fluid_launches": nf.value,
                "boundary_launches": nb.value}


def batch_plan(dims_list, block=1024, nwg=256):
    """Host-only work split of the batched fluid pass: dict with the segments
    ((domain, strip, first plane, end plane) rows), each workgroup's first
    segment, each domain's (rows loaded, output rows, whole-plane flag) and
    the balance (mean / largest workgroup load)."""
    dims = np.ascontiguousarray(np.asarray(dims_list, dtype=np.int32).reshape(-1, 3))
    count = dims.shape[0]
    n = ctypes.c_int(0)
    dp = dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    L = lib()
    st = L.lbm_batch_plan(count, dp, block, nwg, ctypes.byref(n), None, None, None, None)
    if st != OK:
        raise LBMError(st, L.lbm_batch_last_error(None).decode())
    segs = np.zeros((max(n.value, 1), 4), np.uint16)
    first = np.zeros(nwg + 1, np.uint32)
    strips = np.zeros((count, 3), np.int32)
    bal = ctypes.c_double()
    st = L.lbm_batch_plan(count, dp, block, nwg, ctypes.byref(n), segs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                          first.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                          strips.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ctypes.byref(bal))
    if st != OK:
        raise LBMError(st, L.lbm_batch_last_error(None).decode())
    return {"segments": segs[:n.value], "wg_first": first, "strips": strips, "balance": bal.value}


class HomeLBMBatch:
    """Many independent periodic HOME-LBM domains advanced together."""

    def __init__(self, dims_list, taus, masks=None, fmt="q16", stream=None, **options):
        L = lib()
        self.dims = [tuple(int(v) for v in d) for d in dims_list]
        self.count = len(self.dims)
        if len(taus) != self.count:
            raise ValueError("one tau per domain")
        self.fmt = _fmt_code(fmt)
        self.taus = [float(t) for t in taus]
        flat = (ctypes.c_int * (3 * self.count))(*[v for d in self.dims for v in d])
        tau_arr = (ctypes.c_double * self.count)(*self.taus)
        self._masks = []
        mptr = None
        if masks is not None:
            if len(masks) != self.count:
                raise ValueError("one mask (or None) per domain")
            mptr = (ctypes.c_void_p * self.count)()
            for k, m in enumerate(masks):
                if m is None:
                    self._masks.append(None)
                    mptr[k] = None
                    continue
                a = np.ascontiguousarray(m, dtype=np.uint8)
                if a.size != int(np.prod(self.dims[k])):
                    raise ValueError(f"mask {k} must have nx*ny*nz entries")
                self._masks.append(a)
                mptr[k] = a.ctypes.data_as(ctypes.c_void_p)
        h = ctypes.c_void_p()
        self._h = None
        st = L.lbm_batch_create(self.count, flat, tau_arr, mptr, self.fmt, ctypes.byref(h))
        if st != OK:
            raise LBMError(st, L.lbm_batch_last_error(None).decode())
        self._h = h
        if stream is None:
            stream = _torch_stream()
        if stream is not None:
            self._check(L.lbm_batch_set_stream(self._h, ctypes.c_void_p(stream)))
        if options:
            self.set_options(**options)

    def _check(self, st):
        if st != OK:
            msg = lib().lbm_batch_last_error(self._h)
            raise LBMError(st, msg.decode() if msg else "")
        return st

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def options(self) -> Options:
        o = Options()
        self._check(lib().lbm_batch_get_options(self._h, ctypes.byref(o)))
        return o

    def set_options(self, dither_mode=None, seed=None, check_health=None):
        o = self.options()
        if dither_mode is not None:
            o.dither_mode = int(dither_mode)
        if seed is not None:
            o.seed = int(seed) & 0xFFFFFFFF
        if check_health is not None:
            o.check_health = int(bool(check_health))
        self._check(lib().lbm_batch_set_options(self._h, ctypes.byref(o)))

    def _dom(self, d):
        d = int(d)
        if not 0 <= d < self.count:
            raise LBMError(ERR_INVALID_ARG, f"domain index {d} out of range 0..{self.count - 1}")
        return d

    def cells(self, d=None):
        if d is None:
            n = ctypes.c_int64()
            self._check(lib().lbm_batch_total_cells(self._h, ctypes.byref(n)))
            return n.value
        return int(np.prod(self.dims[self._dom(d)]))

    def set_moments(self, d, m):
        p, dev, keep = _ptr(m, np.float32, 10 * self.cells(d))
        self._check(lib().lbm_batch_set_moments(self._h, int(d), p, dev))

    def set_equilibrium(self, d, rho, u):
        n = self.cells(d)
        p1, d1, k1 = _ptr(rho, np.float32, n)
        p2, d2, k2 = _ptr(u, np.float32, 3 * n)
        if d1 != d2:
            raise ValueError("rho and u must both be host arrays or both device tensors")
        self._check(lib().lbm_batch_set_equilibrium(self._h, int(d), p1, p2, d1))

    def get_moments(self, d, out=None):
        shape = (10,) + self.dims[self._dom(d)][::-1]
        if out is None:
            out = np.empty(shape, dtype=np.float32)
        p, dev, keep = _ptr(out, np.float32, int(np.prod(shape)))
        self._check(lib().lbm_batch_get_moments(self._h, int(d), p, dev))
        return out

    def raw_bytes(self, d):
        return lib().lbm_batch_raw_bytes(self._h, int(d))

    def get_raw(self, d, out=None):
        """Raw state of domain d: FP32 (10, nz, ny, nx) float32, Q16 (5, nz, ny, nx) uint32."""
        shape = ((10,) if self.fmt == FP32 else (5,)) + self.dims[self._dom(d)][::-1]
        dt = np.float32 if self.fmt == FP32 else np.uint32
        if out is None:
            out = np.empty(shape, dtype=dt)
        p, dev, keep = _ptr(out, dt, int(np.prod(shape)))
        self._check(lib().lbm_batch_get_raw(self._h, int(d), p, self.raw_bytes(d), dev))
        return out

    def set_raw(self, d, raw):
        dt = np.float32 if self.fmt == FP32 else np.uint32
        n = (10 if self.fmt == FP32 else 5) * self.cells(d)
        p, dev, keep = _ptr(raw, dt, n)
        self._check(lib().lbm_batch_set_raw(self._h, int(d), p, self.raw_bytes(d), dev))

    def step(self, n=1):
        """n steps replayed from captured HIP graphs."""
        self._check(lib().lbm_batch_step(self._h, int(n)))

    def step_eager(self, n=1):
        self._check(lib().lbm_batch_step_eager(self._h, int(n)))

    def profile_steps(self, n):
        f, b = ctypes.c_double(), ctypes.c_double()
        self._check(lib().lbm_batch_profile_steps(self._h, int(n), ctypes.byref(f), ctypes.byref(b)))
        return {"fluid_ms": f.value, "boundary_ms": b.value, "steps": int(n)}

    def synchronize(self):
        self._check(lib().lbm_batch_synchronize(self._h))

    @property
    def step_count(self):
        t = ctypes.c_uint64()
        self._check(lib().lbm_batch_get_step_count(self._h, ctypes.byref(t)))
        return t.value

    @step_count.setter
    def step_count(self, t):
        self._check(lib().lbm_batch_set_step_count(self._h, int(t)))

    def boundary_counts(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().lbm_batch_boundary_counts(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def memory_bytes(self):
        s, t = ctypes.c_size_t(), ctypes.c_size_t()
        self._check(lib().lbm_batch_memory_bytes(self._h, ctypes.byref(s), ctypes.byref(t)))
        return s.value, t.value

    def check(self):
        bad = ctypes.c_uint64()
        st = lib().lbm_batch_check(self._h, ctypes.byref(bad))
        if st not in (OK, ERR_UNSTABLE):
            self._check(st)
        return bad.value

    def tuning(self):
        t = BatchTuning()
        self._check(lib().lbm_batch_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, block, wg_per_cu=1):
        self._check(lib().lbm_batch_set_tuning(self._h, int(block), int(wg_per_cu)))

    def tune(self, cache=None):
        t = BatchTuning()
        self._check(lib().lbm_batch_tune(self._h, None if cache is None else str(cache).encode(), ctypes.byref(t)))
        return t.as_dict()


def _torch_stream():
    """The current torch stream handle if torch with HIP is usable, else None."""
    try:
        import torch
    except ImportError:
        return None
    if not torch.cuda.is_available():
        return None
    return torch.cuda.current_stream().cuda_stream
