"""The oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.

A plain, slow FP64 CPU implementation of the HOME-LBM D3Q27 step
(``homelbm_oracle.cpp``) and this ctypes binding to it.  Only the tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it; the GPU library never does.  Its header lists the paper passages
it follows and the readings it takes where the paper is silent.

Fields are numpy arrays of shape (10, nz, ny, nx) (ten planes, x fastest) in
the stored-moment order rho, jx, jy, jz, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz, with
j = rho u and P = rho S (S the Hermite second moment of Eq. rho_u_stress).
16-bit fields are uint32 arrays of shape (5, nz, ny, nx).

Two numpy modules sit beside it, also test infrastructure: ``d2q9`` (the D2Q9
models and amplification matrices of the paper's 2D von Neumann analysis) and
``stability`` (the same analysis for the 3D step, and speed limits).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "homelbm_oracle.cpp")
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle with g++ -O2 (no fast-math) and OpenMP."""
    tmp = LIB_PATH + ".tmp"
    cmd = ["g++", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c++17", "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int),
        ("ny", ctypes.c_int),
        ("nz", ctypes.c_int),
        ("inflow", ctypes.c_int),
        ("literal_xyz", ctypes.c_int),
        ("tau", ctypes.c_double),
        ("F", ctypes.c_double * 3),
        ("u_in", ctypes.c_double * 3),
        ("wall_rule", ctypes.c_int),
        ("objects", ctypes.POINTER(ctypes.c_double)),
        ("tris", ctypes.POINTER(ctypes.c_float)),
        ("ntris", ctypes.c_int64),
        ("tri_obj", ctypes.POINTER(ctypes.c_uint8)),
    ]


def make_params(dims, tau, F=(0.0, 0.0, 0.0), inflow=False, u_in=(0.0, 0.0, 0.0), literal_xyz=False,
                wall_rule=0, objects=None, triangles=None, tri_obj=None) -> Params:
    """objects: None or a (256, 9) array, row id = center C, velocity V,
    angular velocity W of the solid object with mask value id (R16, R17).
    triangles (T, 9) float32 and tri_obj (T,) uint8: the obstacle meshes of
    wall rule 2 (R26)."""
    nx, ny, nz = (int(d) for d in dims)
    P = Params(nx, ny, nz, int(bool(inflow)), int(bool(literal_xyz)), float(tau),
               (ctypes.c_double * 3)(*[float(v) for v in F]),
               (ctypes.c_double * 3)(*[float(v) for v in u_in]), int(wall_rule), None, None, 0, None)
    if objects is not None:
        obj = np.ascontiguousarray(objects, dtype=np.float64).reshape(256, 9)
        P.object_table = obj  # keeps the table alive as long as the params
        P.objects = obj.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if triangles is not None:
        tr = np.ascontiguousarray(triangles, dtype=np.float32).reshape(-1, 9)
        ob = np.ascontiguousarray(tri_obj, dtype=np.uint8).reshape(-1)
        if ob.size != tr.shape[0]:
            raise ValueError("one object id per triangle")
        P.tri_table, P.obj_table = tr, ob
        P.tris = tr.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        P.ntris = tr.shape[0]
        P.tri_obj = ob.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    return P


_P = ctypes.POINTER
_dp = _P(ctypes.c_double)
_fp = _P(ctypes.c_float)
_u8 = _P(ctypes.c_uint8)
_u32 = _P(ctypes.c_uint32)
_i64 = _P(ctypes.c_int64)
_ip = _P(ctypes.c_int)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_version.restype = ctypes.c_int
        L.orc_lattice.argtypes = [_ip, _dp, _ip]
        L.orc_reconstruct.argtypes = [ctypes.c_double, _dp, _dp, ctypes.c_int, _dp]
        L.orc_project.argtypes = [_dp, _dp, _dp]
        L.orc_collide.argtypes = [ctypes.c_double, _dp, _dp, _dp, ctypes.c_double, _dp]
        L.orc_post_collision_f.argtypes = [_P(Params), _dp, _dp, _dp, _dp]
        L.orc_step.argtypes = [_P(Params), _u8, _dp, _dp, ctypes.c_int]
        L.orc_object_forces.argtypes = [_P(Params), _u8, _dp, _dp]
        L.orc_mesh_links.argtypes = [_P(Params), _u8, _dp, ctypes.c_int64]
        L.orc_mesh_links.restype = ctypes.c_int64
        L.orc_stream_post.argtypes = [_P(Params), _u8, _dp, _dp, ctypes.c_int]
        L.orc_collide_field.argtypes = [_P(Params), _u8, _dp, _dp]
        L.orc_mixed_q16_step.argtypes = [_P(Params), _u8, _u32, _u32, _dp, ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.c_int, ctypes.c_int]
        L.orc_qb_encode.argtypes = [_dp, _u8, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, _u32]
        L.orc_qb_decode.argtypes = [_u32, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _dp]
        L.orc_qb_pack.argtypes = [_u32, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _u32]
        L.orc_qb_step.argtypes = [_P(Params), _u8, _u32, _u32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_step_f32.argtypes = [_P(Params), _u8, _fp, _fp, ctypes.c_int]
        L.orc_step_cs.argtypes = [_P(Params), _u8, _dp, _dp, _dp, _dp, ctypes.c_int]
        L.orc_step_cells.argtypes = [_P(Params), _u8, _dp, ctypes.c_int64, _i64, _dp, ctypes.c_int]
        L.orc_pcg_hash.argtypes = [ctypes.c_uint32]
        L.orc_pcg_hash.restype = ctypes.c_uint32
        L.orc_dither.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, _dp, _u32]
        L.orc_encode_one.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double]
        L.orc_encode_one.restype = ctypes.c_uint32
        L.orc_encode_one_b.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int]
        L.orc_encode_one_b.restype = ctypes.c_uint32
        L.orc_decode_one.argtypes = [ctypes.c_uint32, ctypes.c_int]
        L.orc_decode_one.restype = ctypes.c_double
        L.orc_q16_encode.argtypes = [_dp, _u8, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, _u32]
        L.orc_q16_decode.argtypes = [_u32, ctypes.c_int64, _dp]
        L.orc_q16_step.argtypes = [_P(Params), _u8, _u32, _u32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                   ctypes.c_int]
        L.orc_q16_step_cells.argtypes = [_P(Params), _u8, _u32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                         ctypes.c_int64, _i64, _u32, ctypes.c_int]
        L.orc_adjoint_step.argtypes = [_P(Params), _u8, _dp, _dp, _dp, ctypes.c_int]
        L.orc_adjoint_step_cells.argtypes = [_P(Params), _u8, _dp, _dp, ctypes.c_int64, _i64, _dp, ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(t)


def _mask_ptr(mask):
    if mask is None:
        return None, None
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    return m, _ptr(m, _u8)


def default_threads() -> int:
    """OMP_NUM_THREADS when set, else the CPUs this process may run on."""
    try:
        n = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        n = 0
    if n <= 0:
        try:
            n = len(os.sched_getaffinity(0))
        except (AttributeError, OSError):
            n = os.cpu_count() or 1
    return max(1, n)


# ---------------------------------------------------------------- lattice ---

def lattice():
    """(c[27,3] int, w[27], opp[27]) of the D3Q27 lattice, i = (cx+1)+3(cy+1)+9(cz+1)."""
    c = np.zeros(81, dtype=np.int32)
    w = np.zeros(27)
    opp = np.zeros(27, dtype=np.int32)
    lib().orc_lattice(_ptr(c, _ip), _ptr(w, _dp), _ptr(opp, _ip))
    return c.reshape(27, 3), w, opp


# ------------------------------------------------------------ one cell ------

def reconstruct(rho, u, S6, literal_xyz=False):
    """h(rho, u, S) -> 27 distributions (Eq. three_order_f); S6 = xx, yy, zz, xy, xz, yz."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    S6 = np.ascontiguousarray(S6, dtype=np.float64)
    f = np.zeros(27)
    lib().orc_reconstruct(float(rho), _ptr(u, _dp), _ptr(S6, _dp), int(literal_xyz), _ptr(f, _dp))
    return f


def project(f, F=(0.0, 0.0, 0.0)):
    """Moments (rho, j, P) of 27 distributions (Eq. rho_u_stress)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    m = np.zeros(10)
    lib().orc_project(_ptr(f, _dp), _ptr(F, _dp), _ptr(m, _dp))
    return m


def collide(rho, u, S6, tau, F=(0.0, 0.0, 0.0)):
    """App. A collision -> (rho+, u+ (3), S+ (6))."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    S6 = np.ascontiguousarray(S6, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros(10)
    lib().orc_collide(float(rho), _ptr(u, _dp), _ptr(S6, _dp), _ptr(F, _dp), float(tau), _ptr(out, _dp))
    return out


def post_collision_f(params: Params, m10, m10_im=None):
    """f+ = h(collide(m)) for one cell; complex input gives complex output."""
    re = np.ascontiguousarray(np.real(m10), dtype=np.float64)
    im = None if m10_im is None else np.ascontiguousarray(m10_im, dtype=np.float64)
    fre = np.zeros(27)
    fim = np.zeros(27)
    lib().orc_post_collision_f(ctypes.byref(params), _ptr(re, _dp), None if im is None else _ptr(im, _dp),
                               _ptr(fre, _dp), _ptr(fim, _dp))
    return fre if im is None else fre + 1j * fim


# ------------------------------------------------------------ full grid -----

def _check_field(m, params, dtype=np.float64, comps=10):
    shape = (comps, params.nz, params.ny, params.nx)
    m = np.ascontiguousarray(m, dtype=dtype)
    if m.shape != shape:
        raise ValueError(f"field shape {m.shape} != {shape}")
    return m


def step(params: Params, m, mask=None, nthreads=None):
    """One FP64 step of the whole grid; returns the new (10, nz, ny, nx) field."""
    m = _check_field(m, params)
    out = np.empty_like(m)
    mk, mp = _mask_ptr(mask)
    lib().orc_step(ctypes.byref(params), mp, _ptr(m, _dp), _ptr(out, _dp), nthreads or default_threads())
    return out


def stream_post(params: Params, m_post, mask=None, nthreads=None):
    """Post-stream moments from post-collision moments (the mixed pipeline's
    stream pass, boundary rules included); solid cells get rest."""
    m_post = _check_field(m_post, params, np.float64)
    out = np.empty_like(m_post)
    mk, mp = _mask_ptr(mask)
    lib().orc_stream_post(ctypes.byref(params), mp, _ptr(m_post, _dp), _ptr(out, _dp), nthreads or default_threads())
    return out


def collide_field(params: Params, m, mask=None):
    """Post-collision moments (rho, rho u+, rho S+) of every cell (App. A)."""
    m = _check_field(m, params, np.float64)
    out = np.empty_like(m)
    mk, mp = _mask_ptr(mask)
    lib().orc_collide_field(ctypes.byref(params), mp, _ptr(m, _dp), _ptr(out, _dp))
    return out


def mixed_q16_step(params: Params, w, mask=None, t=0, seed=0, mode=1, nthreads=None):
    """One step of the mixed pipeline on 16-bit post-collision codes:
    returns (codes of the new post-collision state, FP64 post-stream moments)."""
    w = _check_field(w, params, np.uint32, 5)
    out = np.empty_like(w)
    m_ps = np.empty((10,) + w.shape[1:], np.float64)
    mk, mp = _mask_ptr(mask)
    lib().orc_mixed_q16_step(ctypes.byref(params), mp, _ptr(w, _u32), _ptr(out, _u32), _ptr(m_ps, _dp), t, seed, mode,
                             nthreads or default_threads())
    return out, m_ps


def object_forces(params: Params, m, mask):
    """(256, 6) force and torque on each object id during the step from m (R17)."""
    m = _check_field(m, params, np.float64)
    out = np.zeros((256, 6), np.float64)
    mk, mp = _mask_ptr(mask)
    lib().orc_object_forces(ctypes.byref(params), mp, _ptr(m, _dp), _ptr(out, _dp))
    return out


def mesh_links(params: Params, mask):
    """Every link of wall rule 2 (R26): array (n, 7) of cell index, direction
    i, met a triangle (1/0), boundary point p (x, y, z), object id."""
    mk, mp = _mask_ptr(mask)
    n = lib().orc_mesh_links(ctypes.byref(params), mp, None, 0)
    out = np.zeros((max(n, 1), 7))
    lib().orc_mesh_links(ctypes.byref(params), mp, _ptr(out, _dp), n)
    return out[:n]


def run(params: Params, m, nsteps, mask=None, nthreads=None):
    for _ in range(nsteps):
        m = step(params, m, mask, nthreads)
    return m


def step_f32(params: Params, m, mask=None, nthreads=None):
    """The same step instantiated in float (the single-precision floor)."""
    m = _check_field(m, params, np.float32)
    out = np.empty_like(m)
    mk, mp = _mask_ptr(mask)
    lib().orc_step_f32(ctypes.byref(params), mp, _ptr(m, _fp), _ptr(out, _fp), nthreads or default_threads())
    return out


def step_complex(params: Params, m, mask=None, nthreads=1):
    """The same step in complex arithmetic (complex-step derivatives)."""
    m = np.asarray(m)
    re = _check_field(m.real, params)
    im = _check_field(m.imag if np.iscomplexobj(m) else np.zeros_like(re), params)
    ore = np.empty_like(re)
    oim = np.empty_like(re)
    mk, mp = _mask_ptr(mask)
    lib().orc_step_cs(ctypes.byref(params), mp, _ptr(re, _dp), _ptr(im, _dp), _ptr(ore, _dp), _ptr(oim, _dp),
                      nthreads)
    return ore + 1j * oim


def step_cells(params: Params, m, cells, mask=None, nthreads=None):
    """New moments (ncells, 10) at the listed linear cell indices only."""
    m = _check_field(m, params)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((cells.size, 10))
    mk, mp = _mask_ptr(mask)
    lib().orc_step_cells(ctypes.byref(params), mp, _ptr(m, _dp), cells.size, _ptr(cells, _i64), _ptr(out, _dp),
                         nthreads or default_threads())
    return out


def adjoint_step(params: Params, m_t, lam_next, mask=None, nthreads=None):
    """lam_prev = J(m_t)^T lam_next for one step (the per-cell Jacobians on
    nthreads threads)."""
    m_t = _check_field(m_t, params)
    lam_next = _check_field(lam_next, params)
    out = np.zeros_like(m_t)
    mk, mp = _mask_ptr(mask)
    nt = default_threads() if nthreads is None else int(nthreads)
    if lib().orc_adjoint_step(ctypes.byref(params), mp, _ptr(m_t, _dp), _ptr(lam_next, _dp), _ptr(out, _dp), nt) != 0:
        raise ValueError("the oracle's adjoint follows bounce-back walls only (wall_rule 0)")
    return out


def adjoint_step_cells(params: Params, m_t, lam_next, cells, mask=None, nthreads=None):
    """lam_prev = J(m_t)^T lam_next at the given cells only, (ncells, 10):
    the same transpose as adjoint_step, gathered per source cell."""
    m_t = _check_field(m_t, params)
    lam_next = _check_field(lam_next, params)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((cells.size, 10))
    mk, mp = _mask_ptr(mask)
    if lib().orc_adjoint_step_cells(ctypes.byref(params), mp, _ptr(m_t, _dp), _ptr(lam_next, _dp), cells.size,
                                    _ptr(cells, _i64), _ptr(out, _dp),
                                    default_threads() if nthreads is None else int(nthreads)) != 0:
        raise ValueError("the oracle's adjoint follows bounce-back walls only (wall_rule 0)")
    return out


def equilibrium_moments(rho, u):
    """Initial state from (rho, u): j = rho u, P = rho u u (no non-equilibrium part)."""
    dt = np.result_type(np.asarray(rho), np.asarray(u), np.float64)  # complex stays complex
    rho = np.asarray(rho, dtype=dt)
    u = np.asarray(u, dtype=dt)
    m = np.zeros((10,) + rho.shape, dtype=dt)
    m[0] = rho
    for a in range(3):
        m[1 + a] = rho * u[a]
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for p, (a, b) in enumerate(pairs):
        m[4 + p] = rho * u[a] * u[b]
    return m


# ---------------------------------------------------------------- codec -----

Q_LO = np.array([0.8, -0.4, -0.4, -0.4] + [-0.1] * 6)
Q_HI = np.array([1.5, 0.4, 0.4, 0.4] + [0.1] * 6)


def pcg_hash(v: int) -> int:
    return int(lib().orc_pcg_hash(ctypes.c_uint32(v & 0xFFFFFFFF)))


def dither(idx: int, t: int, seed: int, mode: int = 1):
    """(xi[10], (h1, h2)) for cell idx at step t."""
    xi = np.zeros(10)
    h = np.zeros(2, dtype=np.uint32)
    lib().orc_dither(idx & 0xFFFFFFFF, t & 0xFFFFFFFF, seed & 0xFFFFFFFF, mode, _ptr(xi, _dp), _ptr(h, _u32))
    return xi, (int(h[0]), int(h[1]))


def encode_one(m: float, k: int, xi: float = 0.0) -> int:
    return int(lib().orc_encode_one(float(m), int(k), float(xi)))


def qb_encode_one(m: float, k: int, xi: float, b: int) -> int:
    """The b-bit code of one codec variable (R18 ranges and rounding)."""
    return int(lib().orc_encode_one_b(float(m), int(k), float(xi), int(b)))


def decode_one(q: int, k: int) -> float:
    return float(lib().orc_decode_one(int(q), int(k)))


def q16_encode(m, mask=None, t=0, seed=0, mode=0):
    """Encode a (10, nz, ny, nx) field into (5, nz, ny, nx) uint32 words."""
    m = np.ascontiguousarray(m, dtype=np.float64)
    N = int(np.prod(m.shape[1:]))
    out = np.zeros((5,) + m.shape[1:], dtype=np.uint32)
    mk, mp = _mask_ptr(mask)
    lib().orc_q16_encode(_ptr(m, _dp), mp, N, t, seed, mode, _ptr(out, _u32))
    return out


def qb_words(b1, b2):
    return (4 * b1 + 6 * b2 + 31) // 32


def qb_encode(m, b1, b2, mask=None, t=0, seed=0, mode=0):
    """Packed b1 / b2 codes (R18) of a (10, nz, ny, nx) field: (W, nz, ny, nx) words."""
    m = np.ascontiguousarray(m, dtype=np.float64)
    N = int(np.prod(m.shape[1:]))
    out = np.zeros((qb_words(b1, b2),) + m.shape[1:], dtype=np.uint32)
    mk, mp = _mask_ptr(mask)
    if lib().orc_qb_encode(_ptr(m, _dp), mp, N, t, seed, mode, b1, b2, _ptr(out, _u32)) != 0:
        raise ValueError("bit widths must be 2..16")
    return out


def qb_decode(w, b1, b2):
    w = np.ascontiguousarray(w, dtype=np.uint32)
    N = int(np.prod(w.shape[1:]))
    out = np.zeros((10,) + w.shape[1:])
    if lib().orc_qb_decode(_ptr(w, _u32), N, b1, b2, _ptr(out, _dp)) != 0:
        raise ValueError("bit widths must be 2..16")
    return out


def qb_pack(q, b1, b2):
    """(10, ...) integer codes -> (W, ...) packed words."""
    q = np.ascontiguousarray(q, dtype=np.uint32)
    N = int(np.prod(q.shape[1:]))
    out = np.zeros((qb_words(b1, b2),) + q.shape[1:], dtype=np.uint32)
    lib().orc_qb_pack(_ptr(q, _u32), N, b1, b2, _ptr(out, _u32))
    return out


def qb_step(params: Params, w, b1, b2, mask=None, t=0, seed=0, mode=1, nthreads=None):
    """decode -> FP64 step -> encode with the dither of step t, b1 / b2 codes."""
    w = np.ascontiguousarray(w, dtype=np.uint32)
    out = np.empty_like(w)
    mk, mp = _mask_ptr(mask)
    if lib().orc_qb_step(ctypes.byref(params), mp, _ptr(w, _u32), _ptr(out, _u32), t, seed, mode, b1, b2,
                         nthreads or default_threads()) != 0:
        raise ValueError("bit widths must be 2..16")
    return out


def q16_decode(w):
    w = np.ascontiguousarray(w, dtype=np.uint32)
    N = int(np.prod(w.shape[1:]))
    out = np.zeros((10,) + w.shape[1:])
    lib().orc_q16_decode(_ptr(w, _u32), N, _ptr(out, _dp))
    return out


def q16_step(params: Params, w, mask=None, t=0, seed=0, mode=1, nthreads=None):
    """decode -> FP64 step -> encode with the dither of step t."""
    w = _check_field(w, params, np.uint32, 5)
    out = np.empty_like(w)
    mk, mp = _mask_ptr(mask)
    lib().orc_q16_step(ctypes.byref(params), mp, _ptr(w, _u32), _ptr(out, _u32), t, seed, mode,
                       nthreads or default_threads())
    return out


def q16_step_cells(params: Params, w, cells, mask=None, t=0, seed=0, mode=1, nthreads=None):
    w = _check_field(w, params, np.uint32, 5)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((cells.size, 5), dtype=np.uint32)
    mk, mp = _mask_ptr(mask)
    lib().orc_q16_step_cells(ctypes.byref(params), mp, _ptr(w, _u32), t, seed, mode, cells.size,
                             _ptr(cells, _i64), _ptr(out, _u32), nthreads or default_threads())
    return out


def unpack_codes(w):
    """(5, ...) words -> (10, ...) codes, low half first."""
    w = np.asarray(w, dtype=np.uint32)
    q = np.empty((10,) + w.shape[1:], dtype=np.uint32)
    q[0::2] = w & 0xFFFF
    q[1::2] = w >> 16
    return q
