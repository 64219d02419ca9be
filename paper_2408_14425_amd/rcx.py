"""ctypes binding of librcx (``include/rcx.h``).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels. Device arrays are passed as ``torch.Tensor`` (their ``data_ptr()``)
and work is enqueued on the tensor's current HIP stream. Loading fails loudly
when ``librcx.so`` has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librcx.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "rcx.h")

RCX_OK = 0
RCX_W_NOT_CONVERGED = 1
RCX_E_INVALID = -1
RCX_E_UNSUPPORTED = -2
RCX_E_NOMEM = -3
RCX_E_HIP = -4
RCX_E_WORKSPACE = -5
RCX_E_NONFINITE = -6
RCX_T_GEOMETRIC = 0
RCX_T_LENGTH_X4 = 1
RCX_STORE_F32 = 0
RCX_STORE_F16_SCALED = 1
RCX_FLAG_BILINEAR_FIX = 1
RCX_FLAG_CHECK_INPUT = 2
RCX_PROFILE_AUTO = 0
RCX_PROFILE_TABLE = 1


class rcx_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nz", C.c_int32), ("voxel_scale", C.c_double)]


class rcx_params(C.Structure):
    _fields_ = [("n_cascades", C.c_int32), ("c0_dirs", C.c_int32), ("c0_t1", C.c_double),
                ("t_rule", C.c_int32), ("storage", C.c_int32), ("n_incl", C.c_int32),
                ("flags", C.c_uint32)]


class rcx_work(C.Structure):
    _fields_ = [("n_cascades", C.c_int32), ("top_skipped", C.c_int32), ("rays_all", C.c_int64),
                ("rays_nonempty", C.c_int64), ("cell_steps", C.c_int64),
                ("level_rays", C.c_int64 * 16), ("level_steps", C.c_int64 * 16)]


class RcxError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {msg} (status {code})")
        self.code = code


_lib = None


def load() -> C.CDLL:
    """Load librcx.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp, i32, sz = C.c_void_p, C.c_int32, C.c_size_t
    L.rcx_params_default.argtypes = [C.POINTER(rcx_params)]
    L.rcx_plan_create.argtypes = [C.POINTER(rcx_grid), C.POINTER(rcx_params), i32, C.POINTER(vp)]
    L.rcx_plan_workspace_bytes.argtypes = [vp, i32, C.POINTER(sz)]
    L.rcx_plan_work.argtypes = [vp, C.POINTER(rcx_work)]
    L.rcx_plan_set_active_host.argtypes = [vp, vp, C.POINTER(C.c_int64)]
    L.rcx_emergent.argtypes = [vp, i32, vp, vp, C.c_double, C.c_double, i32, vp, vp]
    L.rcx_formal_solve.argtypes = [vp, i32, vp, vp, vp, vp, sz, vp]
    L.rcx_formal_solve_noalloc.argtypes = [vp, i32, vp, vp, vp, vp]
    L.rcx_plan_set_order.argtypes = [vp, i32, i32, i32, i32, i32]
    L.rcx_plan_get_order.argtypes = [vp, i32, C.POINTER(i32)]
    L.rcx_autotune.argtypes = [vp, C.c_char_p, vp]
    L.rcx_plan_destroy.argtypes = [vp]
    L.rcx_plan_set_timing.argtypes = [vp, i32]
    L.rcx_plan_get_timing.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.rcx_error_string.argtypes = [i32]
    L.rcx_error_string.restype = C.c_char_p
    L.rcx_last_error.argtypes = [C.c_char_p, sz]
    for name in ("rcx_params_default", "rcx_plan_create", "rcx_plan_workspace_bytes", "rcx_plan_work",
                 "rcx_formal_solve", "rcx_plan_destroy", "rcx_last_error", "rcx_plan_set_timing",
                 "rcx_plan_get_timing", "rcx_plan_set_active_host", "rcx_emergent", "rcx_formal_solve_noalloc",
                 "rcx_plan_set_order", "rcx_plan_get_order", "rcx_autotune"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def np_shape(a):
    import numpy as np
    return tuple(np.shape(a))


def _check(rc: int, where: str) -> int:
    if rc < 0:
        buf = C.create_string_buffer(512)
        load().rcx_last_error(buf, 512)
        raise RcxError(rc, where, buf.value.decode() or load().rcx_error_string(rc).decode())
    return rc


def _stream_ptr(stream) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _dev_ptr(t, dtype_name: str, what: str) -> int:
    if t is None:
        return 0
    if not t.is_cuda or not t.is_contiguous() or str(t.dtype) != dtype_name:
        raise ValueError(f"{what} must be a contiguous {dtype_name} tensor on the GPU")
    return int(t.data_ptr())


# ------------------------------------------------------------- raw C names


def rcx_params_default() -> rcx_params:
    p = rcx_params()
    _check(load().rcx_params_default(C.byref(p)), "rcx_params_default")
    return p


def rcx_plan_create(grid: rcx_grid, params: rcx_params, max_wave: int) -> int:
    h = C.c_void_p()
    _check(load().rcx_plan_create(C.byref(grid), C.byref(params), int(max_wave), C.byref(h)),
           "rcx_plan_create")
    return h.value


def rcx_plan_workspace_bytes(plan: int, n_wave: int) -> int:
    b = C.c_size_t()
    _check(load().rcx_plan_workspace_bytes(plan, int(n_wave), C.byref(b)), "rcx_plan_workspace_bytes")
    return int(b.value)


def rcx_plan_set_active_host(plan: int, active, n_cascades: int):
    """Flag the active cells ([nz][nx] array, non-zero = active) or, with
    None, make every probe active; returns the flagged probes per cascade."""
    import numpy as np
    counts = (C.c_int64 * max(n_cascades, 1))()
    if active is None:
        _check(load().rcx_plan_set_active_host(plan, None, counts), "rcx_plan_set_active_host")
    else:
        a = np.ascontiguousarray(np.asarray(active) != 0, dtype=np.uint8)
        _check(load().rcx_plan_set_active_host(plan, a.ctypes.data, counts), "rcx_plan_set_active_host")
    return list(counts[:n_cascades])


def rcx_plan_work(plan: int) -> rcx_work:
    w = rcx_work()
    _check(load().rcx_plan_work(plan, C.byref(w)), "rcx_plan_work")
    return w


def rcx_formal_solve(plan: int, n_wave: int, chi, eta, J, workspace=None, stream=None) -> int:
    ws_ptr = _dev_ptr(workspace, "torch.uint8", "workspace")
    ws_bytes = 0 if workspace is None else workspace.numel()
    return _check(load().rcx_formal_solve(plan, int(n_wave), _dev_ptr(chi, "torch.float32", "chi"),
                                          _dev_ptr(eta, "torch.float32", "eta"),
                                          _dev_ptr(J, "torch.float32", "J"), ws_ptr or None,
                                          ws_bytes, _stream_ptr(stream)), "rcx_formal_solve")


def rcx_plan_set_timing(plan: int, enable: bool) -> int:
    return _check(load().rcx_plan_set_timing(plan, int(bool(enable))), "rcx_plan_set_timing")


def rcx_plan_get_timing(plan: int, n_cascades: int):
    """(ms per cascade, ms prep + J, march launches, solves) since the last call."""
    ms = (C.c_double * max(n_cascades, 1))()
    other = C.c_double()
    nl, ns = C.c_int64(), C.c_int64()
    _check(load().rcx_plan_get_timing(plan, ms, C.byref(other), C.byref(nl), C.byref(ns)),
           "rcx_plan_get_timing")
    return list(ms[:n_cascades]), other.value, nl.value, ns.value


def rcx_plan_destroy(plan: int) -> int:
    return _check(load().rcx_plan_destroy(plan), "rcx_plan_destroy")


def rcx_error_string(code: int) -> str:
    return load().rcx_error_string(int(code)).decode()


def rcx_last_error() -> tuple[int, str]:
    buf = C.create_string_buffer(512)
    code = load().rcx_last_error(buf, 512)
    return code, buf.value.decode()


# ------------------------------------------------------------ convenience


@dataclass
class Work:
    n_cascades: int
    top_skipped: bool
    rays_all: int
    rays_nonempty: int
    cell_steps: int
    level_rays: list
    level_steps: list


class Plan:
    """Owns an ``rcx_plan`` for one grid and up to ``max_wave`` wavelengths."""

    def __init__(self, nx: int, nz: int, max_wave: int, voxel_scale: float = 1.0,
                 n_cascades: int = 0, c0_dirs: int = 4, c0_t1: float = 1.5,
                 t_rule: int = RCX_T_GEOMETRIC, storage: int = RCX_STORE_F32, n_incl: int = 1,
                 bilinear_fix: bool = False, check_input: bool = False):
        p = rcx_params_default()
        p.n_cascades, p.c0_dirs, p.c0_t1, p.t_rule, p.storage = n_cascades, c0_dirs, c0_t1, t_rule, storage
        p.n_incl = n_incl
        p.flags = (RCX_FLAG_BILINEAR_FIX if bilinear_fix else 0) | (RCX_FLAG_CHECK_INPUT if check_input else 0)
        self.nx, self.nz, self.max_wave = nx, nz, max_wave
        self.handle = rcx_plan_create(rcx_grid(nx, nz, voxel_scale), p, max_wave)

    def work(self) -> Work:
        w = rcx_plan_work(self.handle)
        n = w.n_cascades
        return Work(n, bool(w.top_skipped), w.rays_all, w.rays_nonempty, w.cell_steps,
                    list(w.level_rays[:n]), list(w.level_steps[:n]))

    def emergent(self, chi, eta, wx: float, wz: float, n_rays: int, I=None, stream=None):
        """Emergent intensity [n_wave][n_rays] of a beam of parallel long
        characteristics of light direction (wx, wz)."""
        import torch
        n_wave = chi.shape[0]
        if I is None:
            I = torch.empty((n_wave, n_rays), dtype=torch.float32, device=chi.device)
        _check(load().rcx_emergent(self.handle, int(n_wave), _dev_ptr(chi, "torch.float32", "chi"),
                                   _dev_ptr(eta, "torch.float32", "eta"), float(wx), float(wz), int(n_rays),
                                   _dev_ptr(I, "torch.float32", "I"), _stream_ptr(stream)), "rcx_emergent")
        return I

    def set_active(self, active):
        """Sparse solve: flag the cells of interest ([nz][nx], non-zero =
        active) or None for the dense solve; returns the flagged probes of
        each cascade."""
        if active is not None and np_shape(active) != (self.nz, self.nx):
            raise ValueError(f"active must have shape ({self.nz}, {self.nx})")
        return rcx_plan_set_active_host(self.handle, active, self.work().n_cascades)

    def set_timing(self, enable: bool):
        rcx_plan_set_timing(self.handle, enable)

    def get_timing(self):
        return rcx_plan_get_timing(self.handle, self.work().n_cascades)

    def workspace_bytes(self, n_wave: int) -> int:
        return rcx_plan_workspace_bytes(self.handle, n_wave)

    def formal_solve(self, chi, eta, J=None, workspace=None, stream=None):
        import torch
        n_wave = chi.shape[0]
        if J is None:
            J = torch.empty_like(chi)
        rcx_formal_solve(self.handle, n_wave, chi, eta, J, workspace, stream)
        return J

    def set_order(self, level: int, tile_p: int, tile_d: int = 32, xcd_chunk: int = 128, shared_walk: int = 0):
        """Launch order of cascade `level` (tile_p = 0: probe-major;
        shared_walk = 1: one cell walk for the 4 rays of a wavefront)."""
        _check(load().rcx_plan_set_order(self.handle, int(level), int(tile_p), int(tile_d), int(xcd_chunk),
                                         int(shared_walk)),
               "rcx_plan_set_order")

    def get_order(self, level: int):
        """(tile_p, tile_d, xcd_chunk, shared_walk) of cascade `level`."""
        out = (C.c_int32 * 4)()
        _check(load().rcx_plan_get_order(self.handle, int(level), out), "rcx_plan_get_order")
        return tuple(out)

    def autotune(self, cache_path=None, stream=None):
        """Tune the launch order of the wide cascades (cached per device and
        geometry in cache_path); returns the orders per cascade."""
        _check(load().rcx_autotune(self.handle, None if cache_path is None else str(cache_path).encode(),
                                   _stream_ptr(stream)), "rcx_autotune")
        return [self.get_order(i) for i in range(self.work().n_cascades)]

    def formal_solve_noalloc(self, chi, eta, J, stream=None):
        """rcx_formal_solve_noalloc: the solve in the library's scratch (no
        allocation; J must be given)."""
        _check(load().rcx_formal_solve_noalloc(self.handle, int(chi.shape[0]), _dev_ptr(chi, "torch.float32", "chi"),
                                               _dev_ptr(eta, "torch.float32", "eta"),
                                               _dev_ptr(J, "torch.float32", "J"), _stream_ptr(stream)),
               "rcx_formal_solve_noalloc")
        return J

    def close(self):
        if getattr(self, "handle", None):
            rcx_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ non-LTE

MAXL, MAXLINE, MAXCONT = 6, 8, 4


class rcx_atom(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("n_lines", C.c_int32), ("n_conts", C.c_int32), ("pad_", C.c_int32),
                ("E_eV", C.c_double * MAXL), ("g", C.c_double * MAXL), ("mass_amu", C.c_double),
                ("line_lower", C.c_int32 * MAXLINE), ("line_upper", C.c_int32 * MAXLINE),
                ("line_lambda_nm", C.c_double * MAXLINE), ("line_f", C.c_double * MAXLINE),
                ("cont_lower", C.c_int32 * MAXCONT), ("cont_upper", C.c_int32 * MAXCONT),
                ("cont_edge_nm", C.c_double * MAXCONT), ("cont_alpha0", C.c_double * MAXCONT),
                ("q_coll", C.c_double * (MAXLINE + MAXCONT))]


def atom_from_dict(d: dict) -> rcx_atom:
    a = rcx_atom()
    a.n_levels = len(d["E_eV"])
    a.n_lines = len(d["lines"])
    a.n_conts = len(d["continua"])
    for i, (e, g) in enumerate(zip(d["E_eV"], d["g"])):
        a.E_eV[i] = e
        a.g[i] = g
    a.mass_amu = d["mass_amu"]
    for k, (lo, hi, lam, f) in enumerate(d["lines"]):
        a.line_lower[k], a.line_upper[k], a.line_lambda_nm[k], a.line_f[k] = lo, hi, lam, f
    for k, (lo, hi, edge, a0) in enumerate(d["continua"]):
        a.cont_lower[k], a.cont_upper[k], a.cont_edge_nm[k], a.cont_alpha0[k] = lo, hi, edge, a0
    for k, q in enumerate(d["q_coll"]):
        a.q_coll[k] = q
    return a


def _load_nlte():
    L = load()
    if getattr(L, "_nlte_bound", False):
        return L
    vp, i32 = C.c_void_p, C.c_int32
    L.rcx_nlte_create.argtypes = [C.POINTER(rcx_grid), C.POINTER(rcx_params), C.POINTER(rcx_atom), i32,
                                  vp, vp, vp, C.POINTER(vp)]
    L.rcx_nlte_set_atmosphere.argtypes = [vp, vp, vp, vp, vp, vp]
    L.rcx_nlte_set_line_profile.argtypes = [vp, i32]
    L.rcx_nlte_set_acceleration.argtypes = [vp, i32, i32, i32]
    L.rcx_nlte_set_charge_conservation.argtypes = [vp, i32]
    L.rcx_nlte_emergent.argtypes = [vp, vp, C.c_double, C.c_double, i32, vp, vp]
    L.rcx_nlte_get_ne.argtypes = [vp, vp, vp]
    L.rcx_nlte_set_pressure_conservation.argtypes = [vp, i32]
    L.rcx_nlte_collisional_ne.argtypes = [vp, i32, vp]
    L.rcx_nlte_set_temperature_cut.argtypes = [vp, C.c_double, C.POINTER(C.c_int64)]
    L.rcx_nlte_lte_populations.argtypes = [vp, vp, vp]
    L.rcx_nlte_formal_solve_rates.argtypes = [vp, vp, vp, vp, vp]
    L.rcx_nlte_stat_eq.argtypes = [vp, vp, vp, C.POINTER(C.c_double), vp]
    L.rcx_nlte_iterate.argtypes = [vp, vp, i32, C.c_double, C.POINTER(C.c_int32), C.POINTER(C.c_double), vp]
    L.rcx_nlte_voigt_eval.argtypes = [vp, i32, vp, vp, vp, vp]
    L.rcx_nlte_voigt_eval_march.argtypes = [vp, i32, vp, vp, vp, vp]
    L.rcx_nlte_dims.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.rcx_nlte_destroy.argtypes = [vp]
    L.rcx_nlte_features.argtypes = [vp, vp, vp, vp, vp]
    L.rcx_nlte_log_departures.argtypes = [vp, vp, vp, vp, vp]
    L.rcx_nlte_warm_start.argtypes = [vp, vp, vp, vp, vp, vp]
    L.rcx_nlte_pops_from_prediction.argtypes = [vp, vp, vp, vp, vp]
    L.rcx_nlte_set_timing.argtypes = [vp, i32]
    L.rcx_nlte_autotune.argtypes = [vp, C.c_char_p, vp]
    L.rcx_nlte_get_timing.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    for n in ("rcx_nlte_set_timing", "rcx_nlte_get_timing", "rcx_nlte_autotune", "rcx_nlte_features", "rcx_nlte_log_departures", "rcx_nlte_warm_start", "rcx_nlte_pops_from_prediction",
              "rcx_nlte_set_charge_conservation", "rcx_nlte_get_ne", "rcx_nlte_emergent", "rcx_nlte_set_pressure_conservation",
              "rcx_nlte_collisional_ne", "rcx_nlte_set_temperature_cut"):
        getattr(L, n).restype = i32
    for n in ("rcx_nlte_create", "rcx_nlte_set_atmosphere", "rcx_nlte_lte_populations",
              "rcx_nlte_formal_solve_rates", "rcx_nlte_stat_eq", "rcx_nlte_iterate", "rcx_nlte_voigt_eval",
              "rcx_nlte_voigt_eval_march",
              "rcx_nlte_dims", "rcx_nlte_destroy"):
        getattr(L, n).restype = i32
    L._nlte_bound = True
    return L


def rcx_nlte_create(grid: rcx_grid, params: rcx_params, atom: rcx_atom, lambda_nm, trans, dnu) -> int:
    import numpy as np
    lam = np.ascontiguousarray(lambda_nm, np.float64)
    tr = np.ascontiguousarray(trans, np.int32)
    dn = np.ascontiguousarray(dnu, np.float64)
    h = C.c_void_p()
    _check(_load_nlte().rcx_nlte_create(C.byref(grid), C.byref(params), C.byref(atom), len(lam), lam.ctypes.data,
                                        tr.ctypes.data, dn.ctypes.data, C.byref(h)), "rcx_nlte_create")
    return h.value


def rcx_nlte_set_acceleration(s: int, order: int, delay: int, period: int) -> int:
    return _check(_load_nlte().rcx_nlte_set_acceleration(s, int(order), int(delay), int(period)),
                  "rcx_nlte_set_acceleration")


def rcx_nlte_set_charge_conservation(s: int, enable: bool) -> int:
    return _check(_load_nlte().rcx_nlte_set_charge_conservation(s, int(bool(enable))),
                  "rcx_nlte_set_charge_conservation")


def rcx_nlte_get_ne(s: int, ne, stream=None) -> int:
    return _check(_load_nlte().rcx_nlte_get_ne(s, _dev_ptr(ne, "torch.float64", "ne"), _stream_ptr(stream)),
                  "rcx_nlte_get_ne")


def rcx_nlte_set_line_profile(s: int, mode: int) -> int:
    return _check(_load_nlte().rcx_nlte_set_line_profile(s, int(mode)), "rcx_nlte_set_line_profile")


def rcx_nlte_set_atmosphere(s: int, T, ne, ntot, vel, stream=None) -> int:
    return _check(_load_nlte().rcx_nlte_set_atmosphere(
        s, _dev_ptr(T, "torch.float64", "T"), _dev_ptr(ne, "torch.float64", "ne"),
        _dev_ptr(ntot, "torch.float64", "ntot"), _dev_ptr(vel, "torch.float32", "vel"), _stream_ptr(stream)),
        "rcx_nlte_set_atmosphere")


def rcx_nlte_lte_populations(s: int, pops, stream=None) -> int:
    return _check(_load_nlte().rcx_nlte_lte_populations(s, _dev_ptr(pops, "torch.float64", "pops"),
                                                        _stream_ptr(stream)), "rcx_nlte_lte_populations")


def rcx_nlte_formal_solve_rates(s: int, pops, rates, J=None, stream=None) -> int:
    return _check(_load_nlte().rcx_nlte_formal_solve_rates(
        s, _dev_ptr(pops, "torch.float64", "pops"), _dev_ptr(rates, "torch.float32", "rates"),
        _dev_ptr(J, "torch.float32", "J") or None, _stream_ptr(stream)), "rcx_nlte_formal_solve_rates")


def rcx_nlte_stat_eq(s: int, rates, pops, stream=None) -> float:
    ch = C.c_double()
    _check(_load_nlte().rcx_nlte_stat_eq(s, _dev_ptr(rates, "torch.float32", "rates"),
                                         _dev_ptr(pops, "torch.float64", "pops"), C.byref(ch), _stream_ptr(stream)),
           "rcx_nlte_stat_eq")
    return ch.value


def rcx_nlte_iterate(s: int, pops, max_iter: int, tol: float, stream=None):
    """Returns (status, iterations, last change); status RCX_OK or RCX_W_NOT_CONVERGED."""
    it, ch = C.c_int32(), C.c_double()
    rc = _check(_load_nlte().rcx_nlte_iterate(s, _dev_ptr(pops, "torch.float64", "pops"), int(max_iter), float(tol),
                                              C.byref(it), C.byref(ch), _stream_ptr(stream)), "rcx_nlte_iterate")
    return rc, it.value, ch.value


def rcx_nlte_voigt_eval(s: int, a, x, out, stream=None) -> int:
    return _check(_load_nlte().rcx_nlte_voigt_eval(s, a.numel(), _dev_ptr(a, "torch.float32", "a"),
                                                   _dev_ptr(x, "torch.float32", "x"),
                                                   _dev_ptr(out, "torch.float32", "out"), _stream_ptr(stream)),
                  "rcx_nlte_voigt_eval")


def rcx_nlte_dims(s: int):
    nl, nt = C.c_int32(), C.c_int32()
    _check(_load_nlte().rcx_nlte_dims(s, C.byref(nl), C.byref(nt)), "rcx_nlte_dims")
    return nl.value, nt.value


def rcx_nlte_destroy(s: int) -> int:
    return _check(_load_nlte().rcx_nlte_destroy(s), "rcx_nlte_destroy")


class Nlte:
    """Owns an ``rcx_nlte`` solver for one non-LTE problem (a
    ``workloads.NlteInput``); arrays live on ``cuda:0``."""

    def __init__(self, inp, n_cascades: int = 0, storage: int = RCX_STORE_F32,
                 line_profile: int = RCX_PROFILE_AUTO, check_input: bool = False, set_atmosphere: bool = True,
                 n_incl: int = 1):
        import torch
        p = rcx_params_default()
        p.n_cascades = n_cascades
        p.storage = storage
        p.n_incl = n_incl
        p.flags = RCX_FLAG_CHECK_INPUT if check_input else 0
        self.inp = inp
        self.handle = rcx_nlte_create(rcx_grid(inp.nx, inp.nz, inp.voxel), p, atom_from_dict(inp.atom),
                                      inp.lambda_nm, inp.trans, inp.dnu)
        rcx_nlte_set_line_profile(self.handle, line_profile)
        self.n_levels, self.n_trans = rcx_nlte_dims(self.handle)
        dev = torch.device("cuda:0")
        self.T = torch.from_numpy(inp.T.astype("float64")).to(dev)
        self.ne = torch.from_numpy(inp.ne.astype("float64")).to(dev)
        self.ntot = torch.from_numpy(inp.ntot.astype("float64")).to(dev)
        self.vel = torch.from_numpy(inp.vel.astype("float32")).to(dev).contiguous()
        if set_atmosphere:
            rcx_nlte_set_atmosphere(self.handle, self.T, self.ne, self.ntot, self.vel)

    def set_atmosphere(self, T, ne, ntot, vel):
        """Set the atmosphere from device arrays (T, ne, ntot FP64 [nz][nx],
        vel FP32 [2][nz][nx])."""
        rcx_nlte_set_atmosphere(self.handle, T, ne, ntot, vel)

    def lte(self):
        import torch
        pops = torch.empty((self.n_levels, self.inp.nz, self.inp.nx), dtype=torch.float64, device="cuda:0")
        rcx_nlte_lte_populations(self.handle, pops)
        return pops

    def formal_solve_rates(self, pops, want_J: bool = False):
        import torch
        rates = torch.empty((self.n_trans, 2, self.inp.nz, self.inp.nx), dtype=torch.float32, device="cuda:0")
        J = torch.empty((self.inp.n_wave, self.inp.nz, self.inp.nx), dtype=torch.float32,
                        device="cuda:0") if want_J else None
        rcx_nlte_formal_solve_rates(self.handle, pops, rates, J)
        return rates, J

    def stat_eq(self, rates, pops) -> float:
        return rcx_nlte_stat_eq(self.handle, rates, pops)

    def iterate(self, pops, max_iter: int, tol: float):
        return rcx_nlte_iterate(self.handle, pops, max_iter, tol)

    def set_acceleration(self, order: int, delay: int = 0, period: int = 1):
        """Ng acceleration of iterate() (order 0 = off)."""
        rcx_nlte_set_acceleration(self.handle, order, delay, period)

    def set_timing(self, enable: bool):
        """Record HIP events around every march launch (measurement)."""
        _check(_load_nlte().rcx_nlte_set_timing(self.handle, int(bool(enable))), "rcx_nlte_set_timing")

    def autotune(self, cache_path=None, stream=None):
        """rcx_nlte_autotune: tune the launch orders of the solver's marches
        (cached per device and geometry in cache_path)."""
        _check(_load_nlte().rcx_nlte_autotune(self.handle, None if cache_path is None else str(cache_path).encode(),
                                              _stream_ptr(stream)), "rcx_nlte_autotune")

    def get_timing(self):
        """{'line': (ms, launches, cell steps x wavelengths), 'continuum':
        (...)} of the march launches recorded since timing was enabled or
        the last call; synchronises on the events."""
        ms = (C.c_double * 2)()
        n = (C.c_int64 * 2)()
        st = (C.c_int64 * 2)()
        _check(_load_nlte().rcx_nlte_get_timing(self.handle, ms, n, st), "rcx_nlte_get_timing")
        return {"line": (ms[0], n[0], st[0]), "continuum": (ms[1], n[1], st[1])}

    def emergent(self, pops, wx: float, wz: float, n_rays: int):
        """Emergent spectra [n_wave][n_rays] at populations pops along the
        beam of parallel long characteristics of light direction (wx, wz)."""
        import torch
        I = torch.empty((self.inp.n_wave, n_rays), dtype=torch.float32, device="cuda")
        _check(_load_nlte().rcx_nlte_emergent(self.handle, _dev_ptr(pops, "torch.float64", "pops"), float(wx),
                                              float(wz), int(n_rays), _dev_ptr(I, "torch.float32", "I"),
                                              _stream_ptr(None)), "rcx_nlte_emergent")
        return I

    def set_charge_conservation(self, enable: bool = True):
        """One Newton-Raphson charge-conservation step after each
        equilibrium step (n_e updated on the device)."""
        rcx_nlte_set_charge_conservation(self.handle, enable)

    def set_pressure_conservation(self, enable: bool = True):
        """Hold the atmosphere's gas pressure by rescaling n_Htot after each
        charge step (needs charge conservation)."""
        _check(_load_nlte().rcx_nlte_set_pressure_conservation(self.handle, int(bool(enable))),
               "rcx_nlte_set_pressure_conservation")

    def set_temperature_cut(self, t_cut: float):
        """Sparse solve: flag the cells with T < t_cut (0 clears); returns
        the flagged probes per cascade."""
        n = 16
        counts = (C.c_int64 * n)()
        _check(_load_nlte().rcx_nlte_set_temperature_cut(self.handle, float(t_cut), counts),
               "rcx_nlte_set_temperature_cut")
        return [c for c in counts if c > 0]

    def collisional_ne(self, n_iter: int = 20):
        """Starting n_e from the collisional rates alone."""
        _check(_load_nlte().rcx_nlte_collisional_ne(self.handle, int(n_iter), _stream_ptr(None)),
               "rcx_nlte_collisional_ne")

    def electron_density(self):
        """The solver's current electron density [ncell], FP64 on the GPU."""
        import torch
        out = torch.empty(self.inp.nx * self.inp.nz, dtype=torch.float64, device="cuda")
        rcx_nlte_get_ne(self.handle, out)
        return out

    def voigt(self, a, x, march: bool = False):
        """H(a, x) from the solver's tables: the full table (features), or
        with march=True the compact table the line march uses."""
        import torch
        out = torch.empty_like(a)
        if march:
            _check(_load_nlte().rcx_nlte_voigt_eval_march(self.handle, a.numel(), _dev_ptr(a, "torch.float32", "a"),
                                                          _dev_ptr(x, "torch.float32", "x"),
                                                          _dev_ptr(out, "torch.float32", "out"), _stream_ptr(None)),
                   "rcx_nlte_voigt_eval_march")
        else:
            rcx_nlte_voigt_eval(self.handle, a, x, out)
        return out

    def features(self, pops, norm=None):
        """Warm-start features [cells][6] (device FP32) at populations pops."""
        import numpy as np
        import torch
        out = torch.empty((self.inp.nx * self.inp.nz, 6), dtype=torch.float32, device="cuda:0")
        nrm = None if norm is None else np.ascontiguousarray(norm, np.float32)
        _check(_load_nlte().rcx_nlte_features(self.handle, _dev_ptr(pops, "torch.float64", "pops"),
                                              None if nrm is None else nrm.ctypes.data,
                                              _dev_ptr(out, "torch.float32", "feat"), _stream_ptr(None)),
               "rcx_nlte_features")
        return out

    def log_departures(self, pops, norm=None):
        import numpy as np
        import torch
        out = torch.empty((self.inp.nx * self.inp.nz, self.n_levels), dtype=torch.float32, device="cuda:0")
        nrm = None if norm is None else np.ascontiguousarray(norm, np.float32)
        _check(_load_nlte().rcx_nlte_log_departures(self.handle, _dev_ptr(pops, "torch.float64", "pops"),
                                                   None if nrm is None else nrm.ctypes.data,
                                                   _dev_ptr(out, "torch.float32", "out"), _stream_ptr(None)),
               "rcx_nlte_log_departures")
        return out

    def warm_start(self, net, feat_norm, targ_norm):
        """Populations predicted by the network (device FP64 [levels][nz][nx])."""
        import numpy as np
        import torch
        pops = torch.empty((self.n_levels, self.inp.nz, self.inp.nx), dtype=torch.float64, device="cuda:0")
        fn = np.ascontiguousarray(feat_norm, np.float32)
        tn = np.ascontiguousarray(targ_norm, np.float32)
        _check(_load_nlte().rcx_nlte_warm_start(self.handle, net.handle, fn.ctypes.data, tn.ctypes.data,
                                                _dev_ptr(pops, "torch.float64", "pops"), _stream_ptr(None)),
               "rcx_nlte_warm_start")
        return pops

    def pops_from_prediction(self, y, targ_norm):
        """Populations (device FP64 [levels][nz][nx]) from standardised
        predicted targets y [cells][levels] (device FP32)."""
        import numpy as np
        import torch
        pops = torch.empty((self.n_levels, self.inp.nz, self.inp.nx), dtype=torch.float64, device="cuda:0")
        tn = np.ascontiguousarray(targ_norm, np.float32)
        _check(_load_nlte().rcx_nlte_pops_from_prediction(self.handle, _dev_ptr(y, "torch.float32", "y"),
                                                          tn.ctypes.data, _dev_ptr(pops, "torch.float64", "pops"),
                                                          _stream_ptr(None)),
               "rcx_nlte_pops_from_prediction")
        return pops

    def close(self):
        if getattr(self, "handle", None):
            rcx_nlte_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ MLP


def _load_mlp():
    L = load()
    if getattr(L, "_mlp_bound", False):
        return L
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.rcx_mlp_create.argtypes = [i32, i32, i32, i32, i32, C.POINTER(vp)]
    L.rcx_mlp_n_params.argtypes = [vp, C.POINTER(i64)]
    L.rcx_mlp_set_params.argtypes = [vp, vp, i64]
    L.rcx_mlp_get_params.argtypes = [vp, vp, i64]
    L.rcx_mlp_forward.argtypes = [vp, vp, vp, i32, vp]
    L.rcx_mlp_gradients.argtypes = [vp, vp, vp, i32, vp, C.POINTER(C.c_float), vp]
    L.rcx_mlp_train_step.argtypes = [vp, vp, vp, i32, C.c_float, C.POINTER(C.c_float), vp]
    L.rcx_mlp_destroy.argtypes = [vp]
    for n in ("rcx_mlp_create", "rcx_mlp_n_params", "rcx_mlp_set_params", "rcx_mlp_get_params", "rcx_mlp_forward",
              "rcx_mlp_gradients", "rcx_mlp_train_step", "rcx_mlp_destroy"):
        getattr(L, n).restype = i32
    L._mlp_bound = True
    return L


def rcx_mlp_create(n_in: int, width: int, depth: int, n_out: int, max_batch: int) -> int:
    h = C.c_void_p()
    _check(_load_mlp().rcx_mlp_create(n_in, width, depth, n_out, max_batch, C.byref(h)), "rcx_mlp_create")
    return h.value


class Mlp:
    """Owns an ``rcx_mlp``."""

    def __init__(self, n_in=6, width=128, depth=4, n_out=4, max_batch=65536):
        self.n_in, self.n_out, self.width, self.depth = n_in, n_out, width, depth
        self.handle = rcx_mlp_create(n_in, width, depth, n_out, max_batch)
        n = C.c_int64()
        _check(_load_mlp().rcx_mlp_n_params(self.handle, C.byref(n)), "rcx_mlp_n_params")
        self.n_params = n.value

    def set_params(self, flat):
        import numpy as np
        f = np.ascontiguousarray(flat, np.float32)
        _check(_load_mlp().rcx_mlp_set_params(self.handle, f.ctypes.data, len(f)), "rcx_mlp_set_params")

    def get_params(self):
        import numpy as np
        f = np.empty(self.n_params, np.float32)
        _check(_load_mlp().rcx_mlp_get_params(self.handle, f.ctypes.data, len(f)), "rcx_mlp_get_params")
        return f

    def forward(self, x, stream=None):
        import torch
        y = torch.empty((x.shape[0], self.n_out), dtype=torch.float32, device=x.device)
        _check(_load_mlp().rcx_mlp_forward(self.handle, _dev_ptr(x, "torch.float32", "x"),
                                           _dev_ptr(y, "torch.float32", "y"), x.shape[0], _stream_ptr(stream)),
               "rcx_mlp_forward")
        return y

    def gradients(self, x, y_ref, stream=None):
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        loss = C.c_float()
        _check(_load_mlp().rcx_mlp_gradients(self.handle, _dev_ptr(x, "torch.float32", "x"),
                                             _dev_ptr(y_ref, "torch.float32", "y_ref"), x.shape[0],
                                             _dev_ptr(g, "torch.float32", "grad"), C.byref(loss),
                                             _stream_ptr(stream)), "rcx_mlp_gradients")
        return loss.value, g

    def train_step(self, x, y_ref, lr: float, stream=None) -> float:
        loss = C.c_float()
        _check(_load_mlp().rcx_mlp_train_step(self.handle, _dev_ptr(x, "torch.float32", "x"),
                                              _dev_ptr(y_ref, "torch.float32", "y_ref"), x.shape[0], float(lr),
                                              C.byref(loss), _stream_ptr(stream)), "rcx_mlp_train_step")
        return loss.value

    def close(self):
        if getattr(self, "handle", None):
            _load_mlp().rcx_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- batches


def _load_batch():
    L = load()
    if getattr(L, "_batch_bound", False):
        return L
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.rcx_batch_create.argtypes = [i32, C.POINTER(rcx_grid), C.POINTER(i32), C.POINTER(rcx_params), C.POINTER(vp)]
    L.rcx_batch_set_order.argtypes = [vp, i32, i32]
    L.rcx_batch_set_graph.argtypes = [vp, i32]
    L.rcx_batch_set_active_host.argtypes = [vp, i32, vp]
    L.rcx_batch_solve.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), vp]
    L.rcx_batch_work.argtypes = [vp, C.POINTER(i64), C.POINTER(i64)]
    L.rcx_batch_launches.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
    L.rcx_batch_autotune.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.c_char_p, C.POINTER(i32), vp]
    L.rcx_batch_destroy.argtypes = [vp]
    for n in ("rcx_batch_create", "rcx_batch_set_order", "rcx_batch_set_graph", "rcx_batch_set_active_host",
              "rcx_batch_solve",
              "rcx_batch_work", "rcx_batch_launches", "rcx_batch_autotune", "rcx_batch_destroy"):
        getattr(L, n).restype = i32
    L._batch_bound = True
    return L


def _ptr_array(ts, what: str):
    arr = (C.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = _dev_ptr(t, "torch.float32", f"{what}[{i}]")
    return arr


class Batch:
    """Owns an ``rcx_batch``: formal solutions of several atmospheres (grids
    ``shapes[a] = (nx, nz)``, ``n_wave[a]`` wavelengths) as one captured
    graph of list-scheduled launches."""

    def __init__(self, shapes, n_wave, voxel_scale=1.0, storage: int = RCX_STORE_F32, c0_t1: float = 1.5,
                 t_rule: int = RCX_T_GEOMETRIC, check_input: bool = False):
        n = len(shapes)
        if len(n_wave) != n:
            raise ValueError("shapes and n_wave differ in length")
        vs = voxel_scale if hasattr(voxel_scale, "__len__") else [voxel_scale] * n
        grids = (rcx_grid * n)(*[rcx_grid(int(nx), int(nz), float(v)) for (nx, nz), v in zip(shapes, vs)])
        nw = (C.c_int32 * n)(*[int(w) for w in n_wave])
        p = rcx_params_default()
        p.storage, p.c0_t1, p.t_rule = storage, c0_t1, t_rule
        p.flags = RCX_FLAG_CHECK_INPUT if check_input else 0
        h = C.c_void_p()
        _check(_load_batch().rcx_batch_create(n, grids, nw, C.byref(p), C.byref(h)), "rcx_batch_create")
        self.handle = h.value
        self.shapes, self.n_wave = [tuple(s) for s in shapes], list(n_wave)

    def set_order(self, tile_probes: int, tile_dirs: int = 32):
        _check(_load_batch().rcx_batch_set_order(self.handle, int(tile_probes), int(tile_dirs)),
               "rcx_batch_set_order")

    def set_graph(self, enable: bool):
        _check(_load_batch().rcx_batch_set_graph(self.handle, int(bool(enable))), "rcx_batch_set_graph")

    def set_active(self, atm: int, active):
        """Sparse atmosphere: flag its cells ([nz][nx], non-zero = active)
        or None for dense."""
        import numpy as np
        L = _load_batch()
        if active is None:
            _check(L.rcx_batch_set_active_host(self.handle, int(atm), None), "rcx_batch_set_active_host")
            return
        nx, nz = self.shapes[atm]
        a = np.ascontiguousarray(np.asarray(active) != 0, dtype=np.uint8)
        if a.shape != (nz, nx):
            raise ValueError(f"active must have shape ({nz}, {nx})")
        _check(L.rcx_batch_set_active_host(self.handle, int(atm), a.ctypes.data), "rcx_batch_set_active_host")

    def work(self):
        r, c = C.c_int64(), C.c_int64()
        _check(_load_batch().rcx_batch_work(self.handle, C.byref(r), C.byref(c)), "rcx_batch_work")
        return r.value, c.value

    def launches(self):
        """(march launches, all launches) one solve enqueues; (0, 0) before
        the first solve."""
        m, a = C.c_int32(), C.c_int32()
        _check(_load_batch().rcx_batch_launches(self.handle, C.byref(m), C.byref(a)), "rcx_batch_launches")
        return m.value, a.value

    def _arrays(self, chi, eta, J):
        import torch
        if J is None:
            J = [torch.empty_like(c) for c in chi]
        if not (len(chi) == len(eta) == len(J) == len(self.shapes)):
            raise ValueError("one chi, eta and J per atmosphere")
        for a, (c, (nx, nz), nw) in enumerate(zip(chi, self.shapes, self.n_wave)):
            if tuple(c.shape) != (nw, nz, nx) or tuple(eta[a].shape) != (nw, nz, nx) or \
                    tuple(J[a].shape) != (nw, nz, nx):
                raise ValueError(f"atmosphere {a}: arrays must be [{nw}][{nz}][{nx}]")
        return J, _ptr_array(chi, "chi"), _ptr_array(eta, "eta"), _ptr_array(J, "J")

    def solve(self, chi, eta, J=None, stream=None):
        J, pc, pe, pj = self._arrays(chi, eta, J)
        _check(_load_batch().rcx_batch_solve(self.handle, pc, pe, pj, _stream_ptr(stream)), "rcx_batch_solve")
        return J

    def autotune(self, chi, eta, J=None, cache_path=None, stream=None) -> int:
        J, pc, pe, pj = self._arrays(chi, eta, J)
        best = C.c_int32()
        path = cache_path.encode() if cache_path else None
        _check(_load_batch().rcx_batch_autotune(self.handle, pc, pe, pj, path, C.byref(best), _stream_ptr(stream)),
               "rcx_batch_autotune")
        return best.value

    def close(self):
        if getattr(self, "handle", None):
            _load_batch().rcx_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
