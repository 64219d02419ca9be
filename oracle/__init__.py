"""FP64 CPU oracle for the radiance-cascades formal solution and the non-LTE
iteration around it (arXiv:2408.14425, Secs. 2-3).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path. It shares no code
with the HIP library; only the seeded input generators are common.

``liboracle.so`` is compiled from ``rc_oracle.c`` by ``__graft_entry__.build()``
(or :func:`build_oracle`).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["rc_oracle.c", "nlte_oracle.c"]


def build_oracle(verbose: bool = False) -> str:
    """Compile the C part of the oracle (plain gcc, FP64, OpenMP; -O3 for
    x86-64-v3, AVX2 and FMA: it is built here and also runs on the GPU
    box's host, whose processor differs, so not -march=native)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Geom(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("nz", C.c_int32), ("n_casc", C.c_int32), ("c0_dirs", C.c_int32),
        ("t1", C.c_double), ("t_rule", C.c_int32), ("bilinear_fix", C.c_int32), ("voxel", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_oracle()
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        gp = C.POINTER(Geom)
        L.ora_t_start.restype = C.c_double
        L.ora_t_start.argtypes = [gp, C.c_int32]
        L.ora_level_dirs.restype = C.c_int32
        L.ora_level_dirs.argtypes = [gp, C.c_int32]
        L.ora_level_px.restype = C.c_int32
        L.ora_level_px.argtypes = [gp, C.c_int32]
        L.ora_level_pz.restype = C.c_int32
        L.ora_level_pz.argtypes = [gp, C.c_int32]
        L.ora_direction.restype = None
        L.ora_direction.argtypes = [gp, C.c_int32, C.c_int32, dp, dp]
        L.ora_segments.restype = C.c_int32
        L.ora_segments.argtypes = [C.c_double] * 6 + [C.c_int32, C.c_int32, ip, ip, dp, C.c_int32]
        L.ora_march.restype = None
        L.ora_march.argtypes = [C.c_int32, dp, dp, dp, dp, dp]
        L.ora_merge.restype = None
        L.ora_merge.argtypes = [C.c_double] * 4 + [dp, dp]
        L.ora_merge_level.restype = None
        L.ora_merge_level.argtypes = [gp, C.c_int32, C.c_int32, dp, dp, dp, dp, C.c_void_p]
        L.ora_formal_solve.restype = C.c_int32
        L.ora_formal_solve.argtypes = [gp, C.c_int32, dp, dp, C.c_void_p, dp, C.c_void_p,
                                       C.POINTER(C.c_int64), C.c_int32]
        L.ora_level_intervals.restype = C.c_int64
        L.ora_level_intervals.argtypes = [gp, C.c_int32, C.c_int32, dp, dp, dp, dp]
        L.ora_lc_solve.restype = C.c_int32
        L.ora_lc_solve.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                   dp, dp, dp, C.c_int32]
        L.ora_lc_points.restype = C.c_int32
        L.ora_lc_points.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_int32, C.c_int32, dp, dp,
                                    C.c_int32, ip, ip, ip, dp, C.c_int32]
        L.ora_num_threads.restype = C.c_int32
        L.ora_emergent.restype = C.c_int32
        L.ora_emergent.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_int32, dp, dp, C.c_double, C.c_double,
                                   C.c_int32, dp, C.c_int32]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def default_cascades(nx: int, nz: int) -> int:
    """Cascade count of a grid when none is given: the smallest k with
    4^k >= max(nx, nz), plus 2. With alpha = 2 the interval starts grow
    as 4^i (Eq. RcScalingLaw, cascade-0 interval 1.5 cells, Sec. 4.5), so
    this is the count at which the top cascade's interval starts at or
    beyond the domain's diagonal: 5 cascades at 64^2, 7 at 1024^2."""
    m = max(int(nx), int(nz))
    k = 0
    while 4 ** k < m:
        k += 1
    return k + 2


def make_geom(nx: int, nz: int, n_casc: int, c0_dirs: int = 4, t1: float = 1.5,
              t_rule: int = 0, voxel: float = 1.0, bilinear_fix: bool = False) -> Geom:
    return Geom(nx, nz, n_casc, c0_dirs, t1, t_rule, int(bool(bilinear_fix)), voxel)


def t_start(g: Geom, i: int) -> float:
    return lib().ora_t_start(C.byref(g), i)


def level_shape(g: Geom, i: int) -> tuple[int, int, int]:
    """(probes z, probes x, directions) of cascade i."""
    L = lib()
    return (L.ora_level_pz(C.byref(g), i), L.ora_level_px(C.byref(g), i),
            L.ora_level_dirs(C.byref(g), i))


def direction(g: Geom, i: int, k: int) -> tuple[float, float]:
    wx, wz = C.c_double(), C.c_double()
    lib().ora_direction(C.byref(g), i, k, C.byref(wx), C.byref(wz))
    return wx.value, wz.value


def segments(cx, cz, wx, wz, ta, tb, nx, nz):
    """Segments of a ray, near -> far: (cell x, cell z, length in cells)."""
    m = nx + nz + 8
    sx = np.zeros(m, np.int32)
    sz = np.zeros(m, np.int32)
    dt = np.zeros(m, np.float64)
    n = lib().ora_segments(cx, cz, wx, wz, ta, tb, nx, nz,
                           sx.ctypes.data_as(C.POINTER(C.c_int32)),
                           sz.ctypes.data_as(C.POINTER(C.c_int32)), _dp(dt), m)
    if n < 0:
        raise RuntimeError("segment buffer overflow")
    return sx[:n].copy(), sz[:n].copy(), dt[:n].copy()


def march(chi, eta, ds):
    """Back-to-front piecewise-constant solution over segments ordered near -> far."""
    chi, eta, ds = _f64(chi), _f64(eta), _f64(ds)
    I, tau = C.c_double(), C.c_double()
    lib().ora_march(len(ds), _dp(chi), _dp(eta), _dp(ds), C.byref(I), C.byref(tau))
    return I.value, tau.value


def merge(near, far):
    """Merge operator on (I, tau) pairs; ``near`` is the interval nearer the probe."""
    I, tau = C.c_double(), C.c_double()
    lib().ora_merge(near[0], near[1], far[0], far[1], C.byref(I), C.byref(tau))
    return I.value, tau.value


def merge_level(g: Geom, i: int, I_i, tau_i, I_up, need=None):
    """Merge cascade i (raw) with merged cascade i+1; arrays [n_wave][pz][px][dirs]."""
    I_i, tau_i = _f64(I_i), _f64(tau_i)
    out = np.zeros_like(I_i)
    up = None if I_up is None else _f64(I_up)
    nm = None if need is None else np.ascontiguousarray(need, dtype=np.uint8)
    lib().ora_merge_level(C.byref(g), i, I_i.shape[0], _dp(I_i), _dp(tau_i),
                          None if up is None else _dp(up), _dp(out),
                          None if nm is None else nm.ctypes.data)
    return out


def formal_solve(chi, eta, n_casc: int, voxel: float = 1.0, c0_dirs: int = 4, t1: float = 1.5,
                 t_rule: int = 0, need=None, want_I0: bool = False, n_threads: int = 0,
                 bilinear_fix: bool = False):
    """RC formal solve in FP64. chi, eta: [n_wave][nz][nx]. Returns J (and the
    merged cascade-0 radiance [n_wave][nz][nx][N_0] if ``want_I0``) and stats
    (rays, non-empty rays, cell steps). ``bilinear_fix``: every cascade below
    the top traces each interval once per bilinear probe of the cascade
    above, to the start of that probe's child cone (Sec. 2.5)."""
    chi, eta = _f64(chi), _f64(eta)
    if chi.ndim == 2:
        chi, eta = chi[None], eta[None]
    nw, nz, nx = chi.shape
    g = make_geom(nx, nz, n_casc, c0_dirs, t1, t_rule, voxel, bilinear_fix)
    J = np.zeros((nw, nz, nx))
    I0 = np.zeros((nw, nz, nx, c0_dirs)) if want_I0 else None
    st = np.zeros(3, np.int64)
    nm = None if need is None else np.ascontiguousarray(need, dtype=np.uint8)
    rc = lib().ora_formal_solve(C.byref(g), nw, _dp(chi), _dp(eta),
                                None if nm is None else nm.ctypes.data, _dp(J),
                                None if I0 is None else I0.ctypes.data,
                                st.ctypes.data_as(C.POINTER(C.c_int64)), n_threads)
    if rc != 0:
        raise RuntimeError(f"ora_formal_solve failed ({rc})")
    out = {"J": J, "rays": int(st[0]), "nonempty": int(st[1]), "steps": int(st[2])}
    if want_I0:
        out["I0"] = I0
    return out


def formal_solve_sparse(chi, eta, n_casc: int, active, **kw):
    """Sparse formal solve (Sec. 3.5): ``active`` [nz][nx] flags the cells
    of interest, which are the flagged probes of cascade 0; the probes of
    cascade i+1 that are bilinear parents of flagged probes of cascade i are
    flagged in turn up to the top cascade (the dependency cone of the
    flagged cells), only flagged probes' intervals are computed, and cells
    not flagged are transparent with no emission. J is 0 at cells not
    flagged. Returns the ``formal_solve`` dictionary."""
    chi, eta = _f64(chi), _f64(eta)
    if chi.ndim == 2:
        chi, eta = chi[None], eta[None]
    m = np.asarray(active, dtype=bool)
    out = formal_solve(np.where(m, chi, 0.0), np.where(m, eta, 0.0), n_casc, need=m.astype(np.uint8), **kw)
    out["J"][:, ~m] = 0.0
    return out


def radau_inclinations(n: int):
    """Gauss-Radau rule on mu = cos(angle to the invariant y axis) in [0, 1]
    with the node mu = 0 (the in-plane ray) fixed (Sec. 3.1: eight
    inclined rays per flatland ray integrate one hemisphere, the other being
    its mirror image in a y-invariant model). Nodes: 0 and the roots of
    (P_{n-1} + P_n)(x) / (1 + x), x = 2 mu - 1; weights 2/n^2 and
    (1 - x) / (n^2 P_{n-1}(x)^2), halved for [0, 1]. n = 1 is flatland."""
    from numpy.polynomial import legendre as leg
    if n == 1:
        return np.array([0.0]), np.array([1.0])
    c = np.zeros(n + 1)
    c[n - 1] = c[n] = 1.0
    r = np.sort(np.real(leg.legroots(c)))
    r = r[np.abs(r + 1.0) > 1e-9]
    dc = leg.legder(c)
    for _ in range(3):  # polish the companion-matrix roots
        r = r - leg.legval(r, c) / leg.legval(r, dc)
    pn1 = leg.legval(r, np.eye(n)[n - 1])
    x = np.concatenate([[-1.0], r])
    w = np.concatenate([[2.0 / n ** 2], (1.0 - r) / (n ** 2 * pn1 ** 2)])
    return 0.5 * (x + 1.0), 0.5 * w


def formal_solve_inclined(chi, eta, n_casc: int, n_incl: int, voxel: float = 1.0, **kw):
    """J of the 2D-invariant formal solution: sum over the inclinations of
    the flatland solution whose path per projected cell is 1/sin(theta)
    = 1/sqrt(1 - mu^2) times longer (the same x-z projection), weighted by
    the Gauss-Radau weights."""
    mu, w = radau_inclinations(n_incl)
    J = None
    for m in range(n_incl):
        Jm = formal_solve(chi, eta, n_casc, voxel=voxel / np.sqrt(1.0 - mu[m] ** 2), **kw)["J"]
        J = w[m] * Jm if J is None else J + w[m] * Jm
    return J


def level_intervals(g: Geom, i: int, chi, eta):
    """Raw (I, tau) of every interval of cascade i; [n_wave][pz][px][dirs]."""
    chi, eta = _f64(chi), _f64(eta)
    if chi.ndim == 2:
        chi, eta = chi[None], eta[None]
    pz, px, nd = level_shape(g, i)
    I = np.zeros((chi.shape[0], pz, px, nd))
    tau = np.zeros_like(I)
    lib().ora_level_intervals(C.byref(g), i, chi.shape[0], _dp(chi), _dp(eta), _dp(I), _dp(tau))
    return I, tau


def lc_solve(chi, eta, M: int, voxel: float = 1.0, n_threads: int = 0):
    """Long-characteristics J with M uniformly spaced directions per cell."""
    chi, eta = _f64(chi), _f64(eta)
    if chi.ndim == 2:
        chi, eta = chi[None], eta[None]
    nw, nz, nx = chi.shape
    J = np.zeros((nw, nz, nx))
    lib().ora_lc_solve(nx, nz, voxel, M, nw, _dp(chi), _dp(eta), _dp(J), n_threads)
    return J


def lc_points(chi, eta, M: int, pts, voxel: float = 1.0, n_threads: int = 0):
    """Long-characteristics J at selected (x, z, wavelength index) triples."""
    chi, eta = _f64(chi), _f64(eta)
    if chi.ndim == 2:
        chi, eta = chi[None], eta[None]
    nw, nz, nx = chi.shape
    pts = np.asarray(pts, dtype=np.int32).reshape(-1, 3)
    px, pz, pl = (np.ascontiguousarray(pts[:, j]) for j in range(3))
    J = np.zeros(len(pts))
    ip = C.POINTER(C.c_int32)
    lib().ora_lc_points(nx, nz, voxel, M, nw, _dp(chi), _dp(eta), len(pts),
                        px.ctypes.data_as(ip), pz.ctypes.data_as(ip), pl.ctypes.data_as(ip),
                        _dp(J), n_threads)
    return J


def emergent(chi, eta, wx: float, wz: float, n_rays: int, voxel: float = 1.0, n_threads: int = 0):
    """Emergent intensity [n_wave][n_rays] of a beam of parallel long
    characteristics of light direction (wx, wz) (Sec. 3.9), ray j at offset
    j + 1/2 - n_rays/2 cells across the beam from the domain centre."""
    chi, eta = _f64(chi), _f64(eta)
    if chi.ndim == 2:
        chi, eta = chi[None], eta[None]
    nw, nz, nx = chi.shape
    I = np.zeros((nw, n_rays))
    rc = lib().ora_emergent(nx, nz, voxel, nw, _dp(chi), _dp(eta), wx, wz, n_rays, _dp(I), n_threads)
    if rc != 0:
        raise RuntimeError("ora_emergent failed")
    return I


def num_threads() -> int:
    return int(lib().ora_num_threads())
