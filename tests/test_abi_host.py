"""The C-ABI library without a GPU: exported symbols, host validation paths and
the host build of the device special functions."""
import ctypes
import os
import re

import numpy as np
import pytest
from scipy import special

from paper_1712_07206_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hsbuild.h")).read()
    return sorted(set(re.findall(r"\b(hsbuild_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = N.lib()
    names = declared_functions()
    assert set(names) == set(N.EXPORTS)
    for name in names:
        assert hasattr(L, name), name


def _config(**over):
    rng = np.random.default_rng(0)
    keep = {}
    l_max = over.pop("l_max", 3)
    n_types = over.pop("n_types", 2)
    atom_type = np.asarray(over.pop("atom_type", [0, 0, 1]), dtype=np.int32)
    radial = over.pop("radial", rng.uniform(0.5, 1.5, (n_types, l_max + 1, 4)))
    radial = np.ascontiguousarray(radial, dtype=np.float64)
    udot = np.ascontiguousarray(over.pop("udot", np.full((n_types, l_max + 1), 0.05)))
    r_mt = np.ascontiguousarray(over.pop("r_mt", np.full(n_types, 1.5)))
    cfg = N.HsbConfig()
    cfg.n_types = n_types
    cfg.n_atoms = len(atom_type)
    cfg.l_max = l_max
    cfg.max_ng = over.pop("max_ng", 100)
    lat = over.pop("lattice", np.diag([8.0, 8.0, 9.0]).reshape(9))
    for i in range(9):
        cfg.lattice[i] = float(lat[i])
    cfg.atom_type = atom_type.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    cfg.r_mt = r_mt.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    cfg.radial = radial.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    cfg.udot_norm2 = udot.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    cfg.precision = over.pop("precision", N.HSB_FP64)
    cfg.n_slices = over.pop("n_slices", 0)
    assert not over
    keep.update(atom_type=atom_type, radial=radial, udot=udot, r_mt=r_mt)
    return cfg, keep


def _create(cfg):
    h = ctypes.c_void_p()
    code = N.lib().hsbuild_create(ctypes.byref(cfg), ctypes.byref(h))
    return code, h


def _no_gpu():
    import torch
    return not torch.cuda.is_available()


def test_create_null_arguments():
    h = ctypes.c_void_p()
    assert N.lib().hsbuild_create(None, ctypes.byref(h)) == N.HSB_ERR_ARG
    assert "null" in N.last_error(None)
    cfg, keep = _config()
    assert N.lib().hsbuild_create(ctypes.byref(cfg), None) == N.HSB_ERR_ARG


@pytest.mark.parametrize("field,value", [("n_types", 0), ("n_types", 17), ("n_atoms", 0), ("l_max", -1),
                                         ("l_max", 13), ("max_ng", 0), ("precision", 7)])
def test_create_rejects_out_of_range(field, value):
    cfg, keep = _config()
    setattr(cfg, field, value)
    code, h = _create(cfg)
    assert code == N.HSB_ERR_ARG
    assert N.last_error(None)


@pytest.mark.parametrize("precision", [N.HSB_SPLIT_FP16, N.HSB_SPLIT_BF16, N.HSB_SPLIT_INT8])
@pytest.mark.parametrize("n_slices", [0, 2, 7])
def test_create_rejects_split_slice_count(precision, n_slices):
    cfg, keep = _config(precision=precision, n_slices=n_slices)
    assert _create(cfg)[0] == N.HSB_ERR_ARG
    assert "n_slices" in N.last_error(None)


@pytest.mark.parametrize("precision", [N.HSB_SPLIT_CRT, N.HSB_SPLIT_CRT_BF16, N.HSB_SPLIT_CRT_FP16])
@pytest.mark.parametrize("n_moduli", [0, 6, 7, 14, 15, 24])
def test_create_rejects_residue_moduli_count(precision, n_moduli):
    """The residue forms take 8..13 moduli (checked before any device call)."""
    cfg, keep = _config(precision=precision, n_slices=n_moduli)
    assert _create(cfg)[0] == N.HSB_ERR_ARG
    assert "moduli" in N.last_error(None)


@pytest.mark.parametrize("precision", [N.HSB_SPLIT_CRT_FP16 + 1, -1, 99])
def test_create_rejects_unknown_precision(precision):
    cfg, keep = _config(precision=precision, n_slices=5)
    assert _create(cfg)[0] == N.HSB_ERR_ARG
    assert "precision" in N.last_error(None)


def test_create_rejects_unsorted_types():
    cfg, keep = _config(atom_type=[0, 1, 0])
    assert _create(cfg)[0] == N.HSB_ERR_ARG
    assert "non-decreasing" in N.last_error(None)
    cfg, keep = _config(atom_type=[0, 2, 2])
    assert _create(cfg)[0] == N.HSB_ERR_ARG


def test_create_rejects_singular_wronskian():
    radial = np.full((2, 4, 4), 1.0)  # u udot' - udot u' = 0
    cfg, keep = _config(radial=radial)
    assert _create(cfg)[0] == N.HSB_ERR_NUMERIC
    assert "Wronskian" in N.last_error(None)


def test_create_rejects_bad_radius_and_norm():
    cfg, keep = _config(r_mt=np.array([1.0, -1.0]))
    assert _create(cfg)[0] == N.HSB_ERR_ARG
    cfg, keep = _config(udot=np.full((2, 4), -0.1))
    assert _create(cfg)[0] == N.HSB_ERR_ARG
    cfg, keep = _config(lattice=np.zeros(9))
    assert _create(cfg)[0] == N.HSB_ERR_ARG


@pytest.mark.skipif(not _no_gpu(), reason="checks the no-device path")
def test_create_without_device_reports_device_error():
    cfg, keep = _config()
    code, h = _create(cfg)
    assert code == N.HSB_ERR_DEVICE
    assert N.last_error(None)


def test_null_handle_entry_points():
    L = N.lib()
    assert L.hsbuild_workspace_bytes(None, 0, 1, (ctypes.c_int32 * 1)(10)) == 0
    kf = (ctypes.c_double * 3)(0, 0, 0)
    assert L.hsbuild_forward(None, kf, 1, None, None, None, None, None, None, 0, None) == N.HSB_ERR_ARG
    assert L.hsbuild_coefficients(None, kf, 1, None, None, None, None, 0, None) == N.HSB_ERR_ARG
    assert L.hsbuild_forward_static(None, kf, 1, None, None, None, None, None, None) == N.HSB_ERR_ARG
    L.hsbuild_destroy(None)


# ---- host build of the device special functions --------------------------------------

def _mp_bessel(l, x):
    """j_l(x) and j_l'(x) at 40 digits (mpmath), the reference for the host build."""
    import mpmath as mp
    mp.mp.dps = 40
    xm = mp.mpf(float(x))
    if xm == 0:
        return (1.0 if l == 0 else 0.0), (1.0 / 3.0 if l == 1 else 0.0)
    j = lambda n: mp.sqrt(mp.pi / (2 * xm)) * mp.besselj(n + mp.mpf(1) / 2, xm)
    jl = j(l)
    djl = (l * j(l - 1) - (l + 1) * j(l + 1)) / (2 * l + 1) if l > 0 else -j(1)
    env = mp.sqrt(jl ** 2 + (mp.sqrt(mp.pi / (2 * xm)) * mp.bessely(l + mp.mpf(1) / 2, xm)) ** 2)
    return float(jl), float(djl), float(env)


def test_host_bessel_matches_mpmath():
    """Series below x = 2, Miller's recurrence above, x in [0, 12], l <= 12: relative
    error <= 1e-14, plus 2e-15 of the oscillation envelope sqrt(j_l^2 + y_l^2) where
    j_l oscillates (near a zero only the absolute error is meaningful)."""
    L = N.lib()
    lmax = 12
    jl = (ctypes.c_double * (lmax + 1))()
    djl = (ctypes.c_double * (lmax + 1))()
    xs = np.concatenate([[1e-8, 1e-3, 0.4], np.linspace(0.9, 12.0, 75), [1.999999, 2.0, 2.000001, 2 * np.pi]])
    for x in xs:
        assert L.hsbuild_host_bessel(lmax, float(x), jl, djl) == N.HSB_OK
        for l in range(lmax + 1):
            ref, dref, env = _mp_bessel(l, x)
            tol = 1e-14 * abs(ref) + (2e-15 * env if x > l else 0.0)
            assert abs(jl[l] - ref) <= tol + 1e-300, (l, x, jl[l], ref)
            envd = _mp_bessel(max(l - 1, 0), x)[2] + _mp_bessel(l + 1, x)[2]
            dtol = 1e-14 * abs(dref) + (2e-15 * envd if x > l - 1 else 0.0)
            assert abs(djl[l] - dref) <= dtol + 1e-300, (l, x, djl[l], dref)
    assert L.hsbuild_host_bessel(lmax, 0.0, jl, djl) == N.HSB_OK
    assert jl[0] == 1.0 and all(jl[l] == 0.0 for l in range(1, lmax + 1))
    assert abs(djl[1] - 1.0 / 3.0) < 1e-16 and djl[0] == 0.0


def test_host_angular_matches_scipy_harmonics():
    L = N.lib()
    lmax = 12
    out = np.zeros(2 * (lmax + 1) ** 2)
    rng = np.random.default_rng(9)
    vecs = np.concatenate([rng.normal(size=(40, 3)), [[0, 0, 2.0], [0, 0, -1.0], [1e-14, 0, 0], [0, 0, 0],
                                                     [3.0, 0, 0], [0, -2.0, 0]]])
    for v in vecs:
        kv = (ctypes.c_double * 3)(*v)
        assert L.hsbuild_host_angular(lmax, kv, 1.7, out.ctypes.data_as(ctypes.c_void_p)) == N.HSB_OK
        got = out[0::2] + 1j * out[1::2]
        r = np.linalg.norm(v)
        if r < 1e-12:
            theta, phi = 0.0, 0.0
        else:
            theta = np.arccos(np.clip(v[2] / r, -1, 1))
            phi = np.mod(np.arctan2(v[1], v[0]), 2 * np.pi)
        for l in range(lmax + 1):
            for m in range(-l, l + 1):
                ref = 1.7 * (1j ** l) * np.conj(special.sph_harm_y(l, m, theta, phi))
                assert abs(got[l * l + l + m] - ref) <= 1e-14 * 1.7 * np.sqrt((2 * l + 1) / (4 * np.pi)), (v, l, m)


def test_options_null_handle():
    L = N.lib()
    v = ctypes.c_int32()
    assert L.hsbuild_set_option(None, N.HSB_OPT_TILE_GROUP, 4) == N.HSB_ERR_ARG
    assert L.hsbuild_get_option(None, N.HSB_OPT_TILE_GROUP, ctypes.byref(v)) == N.HSB_ERR_ARG
    assert L.hsbuild_set_timing(None, 1) == N.HSB_ERR_ARG
    ms = (ctypes.c_double * N.HSB_TIMING_STAGES)()
    n = ctypes.c_int32()
    assert L.hsbuild_stage_times(None, ms, ctypes.byref(n)) == N.HSB_ERR_ARG


def test_header_is_plain_c(tmp_path):
    """include/hsbuild.h compiles as C99 and C++17 on its own, and a C program
    linked against the library resolves every declared entry point (nothing is
    called: no GPU here)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    names = declared_functions()
    src = tmp_path / "abi.c"
    src.write_text('#include "hsbuild.h"\n#include <stdio.h>\n'
                   "int main(void) {\n  void* p[] = {" + ", ".join("(void*)&%s" % n for n in names) + "};\n"
                   '  printf("%d\\n", (int)(sizeof p / sizeof p[0]));\n  return 0;\n}\n')
    inc = os.path.join(ROOT, "include")
    libdir = os.path.dirname(N.LIB_PATH)
    exe = tmp_path / "abi"
    subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", inc, str(src), "-L", libdir, "-lhsbuild",
                    "-Wl,-rpath," + libdir, "-Wl,--unresolved-symbols=ignore-in-shared-libs", "-o", str(exe)],
                   check=True)
    gxx = shutil.which("g++")
    if gxx is not None:
        subprocess.run([gxx, "-std=c++17", "-Wall", "-Werror", "-x", "c++", "-fsyntax-only", "-I", inc,
                        str(src)], check=True)


@pytest.mark.parametrize("kind,blocks,iters,nbytes,code", [
    (3, 8, 16, 1 << 20, N.HSB_ERR_ARG),                    # unknown kind
    (-1, 8, 16, 1 << 20, N.HSB_ERR_ARG),                   # unknown kind
    (N.HSB_PROBE_INT8_RANDOM, 8, 16, 8 * 256 * 4 - 1, N.HSB_ERR_WORKSPACE),
    (N.HSB_PROBE_FP64, 0, 16, 1 << 20, N.HSB_ERR_ARG),     # no workgroups
    (N.HSB_PROBE_INT8, 8, 0, 1 << 20, N.HSB_ERR_ARG),      # no iterations
    (N.HSB_PROBE_INT8, 8, 24, 1 << 20, N.HSB_ERR_ARG),     # not a multiple of 16
    (N.HSB_PROBE_FP64, 8, 16, 8 * 256 * 8 - 1, N.HSB_ERR_WORKSPACE),
    (N.HSB_PROBE_INT8, 8, 16, 8 * 256 * 4 - 1, N.HSB_ERR_WORKSPACE),
])
def test_mfma_probe_rejects_bad_arguments(kind, blocks, iters, nbytes, code):
    """Checked on the host before any device call (no GPU is touched)."""
    ops = ctypes.c_double(-1.0)
    fake = ctypes.c_void_p(4096)  # never dereferenced: every case fails validation
    assert N.lib().hsbuild_mfma_probe(kind, blocks, iters, fake, nbytes, None, ctypes.byref(ops)) == code
    assert N.last_error(None)
    assert ops.value == -1.0


def test_mfma_probe_rejects_null_buffers():
    ops = ctypes.c_double(0.0)
    assert N.lib().hsbuild_mfma_probe(N.HSB_PROBE_FP64, 8, 16, None, 1 << 20, None, ctypes.byref(ops)) == N.HSB_ERR_ARG
    assert N.lib().hsbuild_mfma_probe(N.HSB_PROBE_FP64, 8, 16, ctypes.c_void_p(4096), 1 << 20, None,
                                      None) == N.HSB_ERR_ARG
