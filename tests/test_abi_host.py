"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid arguments before touching the GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2408_14425_amd import rcx


def _declared_functions():
    text = open(rcx.HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(rcx_[a-z0-9_]+|nlte_[a-z0-9_]+|mlp_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = rcx.load()
    names = _declared_functions()
    assert "rcx_formal_solve" in names and "rcx_plan_create" in names
    for n in names:
        assert hasattr(L, n), f"librcx.so does not export {n}"


def test_error_strings():
    assert rcx.rcx_error_string(0) == "ok"
    assert "invalid" in rcx.rcx_error_string(rcx.RCX_E_INVALID)
    assert "not finite" in rcx.rcx_error_string(rcx.RCX_E_NONFINITE)
    assert rcx.rcx_error_string(-99) == "unknown status code"


def test_header_constants_match_the_binding():
    """The status codes and flags the binding uses are the header's."""
    text = open(rcx.HEADER).read()
    for name in ("RCX_E_INVALID", "RCX_E_UNSUPPORTED", "RCX_E_NOMEM", "RCX_E_HIP", "RCX_E_WORKSPACE",
                 "RCX_E_NONFINITE", "RCX_FLAG_BILINEAR_FIX", "RCX_FLAG_CHECK_INPUT", "RCX_STORE_F32",
                 "RCX_STORE_F16_SCALED"):
        m = re.search(r"#define\s+" + name + r"\s+\(?(-?\d+)u?\)?", text)
        assert m, name
        assert int(m.group(1)) == getattr(rcx, name), name


@pytest.mark.parametrize("nx,nz,mw", [(0, 8, 1), (8, -1, 1), (8, 8, 0)])
def test_plan_create_rejects_bad_sizes(nx, nz, mw):
    p = rcx.rcx_params_default()
    with pytest.raises(rcx.RcxError) as e:
        rcx.rcx_plan_create(rcx.rcx_grid(nx, nz, 1.0), p, mw)
    assert e.value.code == rcx.RCX_E_INVALID


@pytest.mark.parametrize("nx,nz", [(4097, 4096), (1 << 24, 2), (65536, 65536), (2147483647, 2147483647)])
def test_plan_create_rejects_grids_beyond_the_cell_maximum(nx, nz):
    """More than 2^24 cells (the march keeps cell indices in 24-bit products)
    is unsupported, also where nx * nz overflows 32 bits; the check comes
    before any device call, so it runs without a GPU."""
    p = rcx.rcx_params_default()
    with pytest.raises(rcx.RcxError) as e:
        rcx.rcx_plan_create(rcx.rcx_grid(nx, nz, 1.0), p, 1)
    assert e.value.code == rcx.RCX_E_UNSUPPORTED
    code, msg = rcx.rcx_last_error()
    assert code == rcx.RCX_E_UNSUPPORTED and "2^24" in msg


@pytest.mark.parametrize("scale", [0.0, -1.0, float("nan")])
def test_plan_create_rejects_non_positive_voxel_scale(scale):
    p = rcx.rcx_params_default()
    with pytest.raises(rcx.RcxError) as e:
        rcx.rcx_plan_create(rcx.rcx_grid(8, 8, scale), p, 1)
    assert e.value.code == rcx.RCX_E_INVALID


@pytest.mark.parametrize("n_incl", [0, 17])
def test_plan_create_rejects_bad_inclination_counts(n_incl):
    p = rcx.rcx_params_default()
    p.n_incl = n_incl
    with pytest.raises(rcx.RcxError) as e:
        rcx.rcx_plan_create(rcx.rcx_grid(8, 8, 1.0), p, 1)
    assert e.value.code == rcx.RCX_E_INVALID


@pytest.mark.parametrize("flags, n_incl, code", [(4, 1, "RCX_E_INVALID"), (0x80000000, 1, "RCX_E_INVALID"),
                                                 (5, 8, "RCX_E_INVALID"), (7, 1, "RCX_E_INVALID")])
def test_plan_create_rejects_bad_flags(flags, n_incl, code):
    """Unknown flag bits are invalid (with or without the bilinear fix and
    the input check)."""
    p = rcx.rcx_params_default()
    p.flags = flags
    p.n_incl = n_incl
    with pytest.raises(rcx.RcxError) as e:
        rcx.rcx_plan_create(rcx.rcx_grid(8, 8, 1.0), p, 1)
    assert e.value.code == getattr(rcx, code)


def test_sparse_and_emergent_calls_reject_bad_arguments():
    """The sparse, emergent and batch-flag calls validate their arguments
    before touching the device."""
    L = rcx.load()
    assert L.rcx_plan_set_active_host(None, None, None) == rcx.RCX_E_INVALID
    assert L.rcx_emergent(None, 1, None, None, 1.0, 0.0, 4, None, None) == rcx.RCX_E_INVALID
    N = rcx._load_nlte()
    assert N.rcx_nlte_emergent(None, None, 1.0, 0.0, 4, None, None) == rcx.RCX_E_INVALID
    assert N.rcx_nlte_set_temperature_cut(None, 2.5e5, None) == rcx.RCX_E_INVALID
    B = rcx._load_batch()
    assert B.rcx_batch_set_active_host(None, 0, None) == rcx.RCX_E_INVALID


def test_nlte_conservation_calls_reject_null():
    """The charge/pressure conservation and collisional n_e calls reject a
    null solver before touching the device."""
    L = rcx._load_nlte()
    assert L.rcx_nlte_set_charge_conservation(None, 1) == rcx.RCX_E_INVALID
    assert L.rcx_nlte_set_pressure_conservation(None, 1) == rcx.RCX_E_INVALID
    assert L.rcx_nlte_collisional_ne(None, 5, None) == rcx.RCX_E_INVALID
    assert L.rcx_nlte_get_ne(None, None, None) == rcx.RCX_E_INVALID


def test_host_radau_rule_matches_oracle_and_is_exact(tmp_path):
    """The library's inclination rule (host C++, Newton on Legendre
    polynomials) against the oracle's (numpy's Legendre roots), and its
    exactness for polynomials in mu up to degree 2n - 2."""
    import subprocess
    import numpy as np
    import oracle
    src = tmp_path / "radau.cpp"
    src.write_text(
        '#include "incl_quadrature.h"\n#include <cstdio>\n#include <cstdlib>\n'
        "int main(int c, char** v) { std::vector<double> mu, w; rcx::radau_nodes(std::atoi(v[1]), mu, w);"
        ' for (size_t i = 0; i < mu.size(); ++i) std::printf("%.17g %.17g\\n", mu[i], w[i]); return 0; }\n')
    exe = tmp_path / "radau"
    csrc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2408_14425_amd", "csrc")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", csrc, "-o", str(exe), str(src)], check=True)
    for n in (1, 2, 3, 8, 16):
        out = subprocess.run([str(exe), str(n)], check=True, capture_output=True, text=True).stdout
        got = np.array([[float(t) for t in ln.split()] for ln in out.strip().splitlines()])
        mu, w = oracle.radau_inclinations(n)
        np.testing.assert_allclose(got[:, 0], mu, rtol=0, atol=1e-13)
        np.testing.assert_allclose(got[:, 1], w, rtol=1e-10, atol=0)  # numpy roots: ~5e-12 at n = 16
        assert got[0, 0] == 0.0
        for d in range(2 * n - 1):
            assert abs(np.dot(got[:, 1], got[:, 0] ** d) - 1.0 / (d + 1)) < 1e-12


def test_plan_create_rejects_unsupported():
    p = rcx.rcx_params_default()
    p.n_cascades = 17
    with pytest.raises(rcx.RcxError) as e:
        rcx.rcx_plan_create(rcx.rcx_grid(8, 8, 1.0), p, 1)
    assert e.value.code == rcx.RCX_E_INVALID
    code, msg = rcx.rcx_last_error()
    assert code == rcx.RCX_E_INVALID and "n_cascades" in msg


def test_null_arguments_are_rejected():
    L = rcx.load()
    assert L.rcx_plan_create(None, None, 1, None) == rcx.RCX_E_INVALID
    assert L.rcx_formal_solve(None, 1, None, None, None, None, 0, None) == rcx.RCX_E_INVALID
    assert L.rcx_plan_destroy(None) == rcx.RCX_OK
    assert L.rcx_params_default(None) == rcx.RCX_E_INVALID
    rcx._load_nlte()
    assert L.rcx_nlte_set_line_profile(None, rcx.RCX_PROFILE_AUTO) == rcx.RCX_E_INVALID


def _nlte_args():
    from paper_2408_14425_amd import workloads as W
    inp = W.nlte_atmosphere(8, seed=1, n_line=4, n_cont=4)
    return inp, rcx.atom_from_dict(inp.atom)


def test_nlte_create_rejects_bad_wavelength_grouping():
    inp, atom = _nlte_args()
    tr = inp.trans.copy()
    tr[0], tr[-1] = tr[-1], tr[0]
    with pytest.raises(rcx.RcxError) as e:
        rcx.rcx_nlte_create(rcx.rcx_grid(8, 8, inp.voxel), rcx.rcx_params_default(), atom, inp.lambda_nm, tr, inp.dnu)
    assert e.value.code == rcx.RCX_E_INVALID


def test_nlte_create_rejects_unsupported_atom_and_geometry():
    inp, atom = _nlte_args()
    atom.n_levels = 7
    with pytest.raises(rcx.RcxError) as e:
        rcx.rcx_nlte_create(rcx.rcx_grid(8, 8, inp.voxel), rcx.rcx_params_default(), atom, inp.lambda_nm,
                            inp.trans, inp.dnu)
    assert e.value.code == rcx.RCX_E_UNSUPPORTED
    inp, atom = _nlte_args()
    p = rcx.rcx_params_default()
    p.c0_dirs = 8
    with pytest.raises(rcx.RcxError) as e:
        rcx.rcx_nlte_create(rcx.rcx_grid(8, 8, inp.voxel), p, atom, inp.lambda_nm, inp.trans, inp.dnu)
    assert e.value.code == rcx.RCX_E_UNSUPPORTED


def test_nlte_create_rejects_continuum_wavelength_beyond_edge():
    inp, atom = _nlte_args()
    lam = inp.lambda_nm.copy()
    lam[-1] = 95.0  # continuum edge is 91.18 nm
    with pytest.raises(rcx.RcxError) as e:
        rcx.rcx_nlte_create(rcx.rcx_grid(8, 8, inp.voxel), rcx.rcx_params_default(), atom, lam, inp.trans, inp.dnu)
    assert e.value.code == rcx.RCX_E_INVALID


def test_batch_create_rejects_bad_arguments():
    L = rcx._load_batch()
    h = C.c_void_p()
    g = (rcx.rcx_grid * 1)(rcx.rcx_grid(16, 16, 1.0))
    nw = (C.c_int32 * 1)(4)
    p = rcx.rcx_params_default()
    assert L.rcx_batch_create(0, g, nw, C.byref(p), C.byref(h)) == rcx.RCX_E_INVALID
    assert L.rcx_batch_create(1, None, nw, C.byref(p), C.byref(h)) == rcx.RCX_E_INVALID
    p.c0_dirs = 8
    assert L.rcx_batch_create(1, g, nw, C.byref(p), C.byref(h)) == rcx.RCX_E_UNSUPPORTED
    p = rcx.rcx_params_default()
    p.n_cascades = 3
    assert L.rcx_batch_create(1, g, nw, C.byref(p), C.byref(h)) == rcx.RCX_E_UNSUPPORTED
    p = rcx.rcx_params_default()
    p.flags = rcx.RCX_FLAG_BILINEAR_FIX | rcx.RCX_FLAG_CHECK_INPUT
    assert L.rcx_batch_create(1, g, nw, C.byref(p), C.byref(h)) == rcx.RCX_E_UNSUPPORTED
    assert h.value is None
    assert L.rcx_batch_solve(None, None, None, None, None) == rcx.RCX_E_INVALID
    assert L.rcx_batch_set_order(None, 4, 32) == rcx.RCX_E_INVALID
    assert L.rcx_batch_destroy(None) == rcx.RCX_OK
