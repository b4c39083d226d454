"""Host-side checks of the C ABI: the library loads, exports every function
that include/oc.h declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

from paper_2502_14148_amd import oc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:int|const char\*)\s+(oc_\w+)\s*\(", text, re.M))
    return names


def test_header_declares_the_binding_exports():
    assert declared_functions() == set(oc.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(oc._LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_grid_validation_errors():
    lib = oc.load_library()
    g = ctypes.c_void_p()
    bad = oc.GridDesc(100, 32, 32, oc.OC_PERIODIC, 0, 1, 0, 1, 0, 1, oc.OC_RECTILINEAR, 0.0)
    assert lib.oc_grid_create(ctypes.byref(bad), ctypes.byref(g)) == -5
    assert b"unsupported" in lib.oc_last_error()
    bad = oc.GridDesc(32, 32, 32, 7, 0, 1, 0, 1, 0, 1, oc.OC_RECTILINEAR, 0.0)
    assert lib.oc_grid_create(ctypes.byref(bad), ctypes.byref(g)) == -1
    bad = oc.GridDesc(32, 32, 32, oc.OC_BOUNDED, 0, -1, 0, 1, 0, 1, oc.OC_RECTILINEAR, 0.0)
    assert lib.oc_grid_create(ctypes.byref(bad), ctypes.byref(g)) == -1
    assert lib.oc_grid_create(None, ctypes.byref(g)) == -1


def test_workspace_size_and_model_validation():
    lib = oc.load_library()
    g = ctypes.c_void_p()
    gd = oc.GridDesc(32, 32, 16, oc.OC_BOUNDED, 0, 64, 0, 64, -16, 16, oc.OC_RECTILINEAR, 0.0)
    assert lib.oc_grid_create(ctypes.byref(gd), ctypes.byref(g)) == 0
    md = oc.ModelDesc()
    md.precision, md.advection, md.weno_eps, md.weno_q = oc.OC_FP32_MIXED, 1, 1e-15, 2
    md.ntracers, md.buoyancy = 2, 1
    nbytes = ctypes.c_uint64()
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(nbytes)) == 0
    padded = (32 + 6) * (32 + 6) * (16 + 6)
    # two state copies + tendencies for 5 fields in FP32, plus the FP64 spectrum
    assert nbytes.value >= 3 * 5 * padded * 4 + 16 * 32 * 17 * 16
    md.weno_q = 3
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(nbytes)) == -5
    md.weno_q, md.ntracers = 2, 0
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(nbytes)) == -1
    md.ntracers, md.buoyancy = 1, 1
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(nbytes)) == -1
    # a null workspace is refused before any device call
    md.ntracers = 2
    m = ctypes.c_void_p()
    assert lib.oc_model_create(g, ctypes.byref(md), None, 0, ctypes.byref(m)) == -1
    assert lib.oc_grid_destroy(g) == 0


def test_hydrostatic_pairing_is_validated():
    lib = oc.load_library()
    g = ctypes.c_void_p()
    # a lat-lon grid: any multiple of 8 (no FFT constraint), walls in z
    gd = oc.GridDesc(1440, 560, 50, oc.OC_BOUNDED, 0, 360, -70, 140, -3000, 3000, oc.OC_LATLON,
                     6.371e6)
    assert lib.oc_grid_create(ctypes.byref(gd), ctypes.byref(g)) == 0
    md = oc.ModelDesc()
    md.kind, md.precision, md.advection, md.weno_eps, md.weno_q = oc.OC_HYDROSTATIC, 1, 1, 1e-15, 2
    md.ntracers, md.buoyancy, md.depth = 2, 1, 3000.0
    nbytes = ctypes.c_uint64()
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(nbytes)) == 0
    md.kind = oc.OC_NONHYDROSTATIC   # needs a rectilinear grid
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(nbytes)) == -5
    md.kind, md.depth = oc.OC_HYDROSTATIC, 0.0
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(nbytes)) == -1
    assert lib.oc_grid_destroy(g) == 0
    bad = oc.GridDesc(1440, 560, 50, oc.OC_BOUNDED, 0, 360, -70, 170, -3000, 3000, oc.OC_LATLON,
                      6.371e6)
    assert lib.oc_grid_create(ctypes.byref(bad), ctypes.byref(g)) == -1


def test_hydrostatic_field_size_limit():
    """The hydrostatic kernels address a field by 32-bit byte offsets: a
    4096 x 2048 x 64 sector (4102 x 2054 x 70 points with halos) fits in
    FP32 (2.4 GB per field) and is refused in FP64 (4.7 GB)."""
    lib = oc.load_library()
    g = ctypes.c_void_p()
    gd = oc.GridDesc(4096, 2048, 64, oc.OC_BOUNDED, 0, 360, -70, 140, -3000, 3000, oc.OC_LATLON,
                     6.371e6)
    assert lib.oc_grid_create(ctypes.byref(gd), ctypes.byref(g)) == 0
    md = oc.ModelDesc()
    md.kind, md.precision, md.advection, md.weno_eps, md.weno_q = oc.OC_HYDROSTATIC, 1, 1, 1e-15, 2
    md.ntracers, md.buoyancy, md.depth = 2, 1, 3000.0
    nbytes = ctypes.c_uint64()
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(nbytes)) == 0
    md.precision = oc.OC_FP64
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(nbytes)) == -5
    assert "2^32" in lib.oc_last_error().decode()
    assert lib.oc_grid_destroy(g) == 0


def test_ensemble_and_hydrostatic_step_argument_checks():
    lib = oc.load_library()
    nbytes = ctypes.c_uint64()
    assert lib.oc_ensemble_workspace_size(None, 1, ctypes.byref(nbytes)) == -1
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.oc_ensemble_workspace_size(arr, 1, ctypes.byref(nbytes)) == -1
    assert lib.oc_ensemble_workspace_size(arr, 0, ctypes.byref(nbytes)) == -1
    e = ctypes.c_void_p()
    assert lib.oc_ensemble_create(arr, 1, None, 0, 0, ctypes.byref(e)) == -1
    assert lib.oc_ensemble_step(None, ctypes.c_double(1.0), 1, None) == -1
    assert lib.oc_ensemble_destroy(None) == 0
    w = (ctypes.c_double * 1)(1.0)
    assert lib.oc_hydrostatic_step(None, ctypes.c_double(600.0), 30, 1, w, 1, None) == -1


def _faces(vals):
    arr = (ctypes.c_double * len(vals))(*vals)
    return arr, ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))


def test_stretched_grid_validation():
    """z faces: strictly increasing, from z0 to z0 + lz, bounded z, 4..256
    levels (any count: the tridiagonal solve replaces the z transform);
    implicit vertical diffusion needs walls; the learned closure a uniform z."""
    from paper_2502_14148_amd import inputs
    lib = oc.load_library()
    g = ctypes.c_void_p()
    zf = inputs.stretched_faces(50, 100.0, -100.0, 1.5)
    keep, ptr = _faces(zf)
    gd = oc.GridDesc(32, 32, 50, oc.OC_BOUNDED, 0, 64, 0, 64, -100, 100, oc.OC_RECTILINEAR, 0.0)
    gd.z_faces = ptr
    assert lib.oc_grid_create(ctypes.byref(gd), ctypes.byref(g)) == 0
    md = oc.ModelDesc()
    md.precision, md.advection, md.weno_eps, md.weno_q = oc.OC_FP32_MIXED, 1, 1e-15, 2
    md.ntracers, md.buoyancy, md.implicit_z = 2, 1, 1
    nbytes = ctypes.c_uint64()
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(nbytes)) == 0
    md.closure = 1
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(nbytes)) == -5
    md.closure, md.implicit_z = 0, 2
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(nbytes)) == -1
    assert lib.oc_grid_destroy(g) == 0
    # faces out of order, not spanning the domain, periodic z, too many levels
    bad = list(zf)
    bad[10], bad[11] = bad[11], bad[10]
    keep, gd.z_faces = _faces(bad)
    assert lib.oc_grid_create(ctypes.byref(gd), ctypes.byref(g)) == -1
    keep, gd.z_faces = _faces([z + 1.0 for z in zf])
    assert lib.oc_grid_create(ctypes.byref(gd), ctypes.byref(g)) == -1
    keep, gd.z_faces = _faces(zf)
    gd.topology_z = oc.OC_PERIODIC
    assert lib.oc_grid_create(ctypes.byref(gd), ctypes.byref(g)) == -5
    gd.topology_z, gd.nz = oc.OC_BOUNDED, 300
    keep, gd.z_faces = _faces(inputs.stretched_faces(300, 100.0, -100.0))
    assert lib.oc_grid_create(ctypes.byref(gd), ctypes.byref(g)) == -5
    # implicit vertical diffusion with a periodic z
    gd = oc.GridDesc(32, 32, 32, oc.OC_PERIODIC, 0, 1, 0, 1, 0, 1, oc.OC_RECTILINEAR, 0.0)
    assert lib.oc_grid_create(ctypes.byref(gd), ctypes.byref(g)) == 0
    md.implicit_z, md.buoyancy = 1, 0
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(nbytes)) == -5
    assert lib.oc_grid_destroy(g) == 0


def test_les_validation():
    lib = oc.load_library()
    g = ctypes.c_void_p()
    gd = oc.GridDesc(32, 32, 16, oc.OC_BOUNDED, 0, 64, 0, 64, -16, 16, oc.OC_RECTILINEAR, 0.0)
    assert lib.oc_grid_create(ctypes.byref(gd), ctypes.byref(g)) == 0
    md = oc.ModelDesc()
    md.precision, md.advection, md.weno_eps, md.weno_q = oc.OC_FP32_MIXED, 1, 1e-15, 2
    md.ntracers, md.buoyancy = 2, 1
    md.les, md.les_c, md.les_cb, md.les_pr = 1, 0.16, 1.0, 1.0
    nbytes = ctypes.c_uint64()
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(nbytes)) == 0
    plain = ctypes.c_uint64()
    md.les = 0
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(plain)) == 0
    assert nbytes.value > plain.value          # viscosity and closure-tendency buffers
    md.les = 3
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(nbytes)) == -1
    md.les, md.les_c = 2, 0.0
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(nbytes)) == -1
    md.les_c, md.closure = 1.0 / 12.0, 1
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(nbytes)) == -5
    assert lib.oc_grid_destroy(g) == 0


def test_weno_order_validation():
    """WENO7/9 widen the halo (the workspace grows); the hydrostatic model
    takes WENO5 only; unknown schemes are refused."""
    lib = oc.load_library()
    g = ctypes.c_void_p()
    gd = oc.GridDesc(32, 32, 16, oc.OC_BOUNDED, 0, 64, 0, 64, -16, 16, oc.OC_RECTILINEAR, 0.0)
    assert lib.oc_grid_create(ctypes.byref(gd), ctypes.byref(g)) == 0
    md = oc.ModelDesc()
    md.precision, md.weno_eps, md.weno_q = oc.OC_FP32_MIXED, 1e-15, 2
    md.ntracers, md.buoyancy = 2, 1
    sizes = {}
    for name in ("weno5z", "weno7z", "weno7_linear", "weno9z", "weno9_linear"):
        md.advection = oc.ADVECTION[name]
        n = ctypes.c_uint64()
        assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(n)) == 0, name
        sizes[name] = n.value
    assert sizes["weno5z"] < sizes["weno7z"] == sizes["weno7_linear"] < sizes["weno9z"]
    md.advection = 7
    n = ctypes.c_uint64()
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(n)) == -1
    md.advection, md.weno_q = oc.ADVECTION["weno9z"], 3
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(n)) == -5
    assert lib.oc_grid_destroy(g) == 0
    gl = ctypes.c_void_p()
    gdl = oc.GridDesc(64, 32, 8, oc.OC_BOUNDED, 0, 64, -40, 80, -3000, 3000, oc.OC_LATLON,
                      6.371e6)
    assert lib.oc_grid_create(ctypes.byref(gdl), ctypes.byref(gl)) == 0
    mh = oc.ModelDesc()
    mh.kind, mh.precision, mh.weno_eps, mh.weno_q = oc.OC_HYDROSTATIC, oc.OC_FP32_MIXED, 1e-15, 2
    mh.ntracers, mh.buoyancy, mh.depth = 2, 1, 3000.0
    mh.advection = oc.ADVECTION["weno5z"]
    assert lib.oc_model_workspace_size(gl, ctypes.byref(mh), ctypes.byref(n)) == 0
    mh.advection = oc.ADVECTION["weno7z"]
    assert lib.oc_model_workspace_size(gl, ctypes.byref(mh), ctypes.byref(n)) == -5
    assert lib.oc_grid_destroy(gl) == 0


def test_immersed_validation():
    """An immersed boundary reserves the mask and the iteration's vectors;
    it needs WENO5 (or none), a uniform z, no implicit diffusion, LES or
    learned closure, and sane iteration limits."""
    lib = oc.load_library()
    g = ctypes.c_void_p()
    gd = oc.GridDesc(32, 32, 16, oc.OC_BOUNDED, 0, 64, 0, 64, -16, 16, oc.OC_RECTILINEAR, 0.0)
    assert lib.oc_grid_create(ctypes.byref(gd), ctypes.byref(g)) == 0
    md = oc.ModelDesc()
    md.precision, md.advection, md.weno_eps, md.weno_q = oc.OC_FP32_MIXED, 1, 1e-15, 2
    md.ntracers, md.buoyancy = 2, 1
    plain, imm = ctypes.c_uint64(), ctypes.c_uint64()
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(plain)) == 0
    md.immersed, md.cg_tol, md.cg_maxiter = 1, 1e-13, 200
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(imm)) == 0
    assert imm.value >= plain.value + 4 * 32 * 32 * 16 * 8     # four FP64 vectors at least
    n = ctypes.c_uint64()
    for field, bad, rc in (("cg_tol", 0.0, -1), ("cg_maxiter", 0, -1), ("immersed", 2, -1),
                           ("advection", oc.ADVECTION["weno9z"], -5), ("implicit_z", 1, -5),
                           ("les", 1, -5), ("closure", 1, -5)):
        good = getattr(md, field)
        setattr(md, field, bad)
        if field == "les":
            md.les_c, md.les_cb, md.les_pr = 0.16, 1.0, 1.0
        assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(n)) == rc, field
        setattr(md, field, good)
    assert lib.oc_grid_destroy(g) == 0
    # a stretched z is refused
    zf = (ctypes.c_double * 17)(*[-16.0 + 16.0 * (k / 16) ** 1.3 for k in range(17)])
    gs = oc.GridDesc(32, 32, 16, oc.OC_BOUNDED, 0, 64, 0, 64, -16, 16, oc.OC_RECTILINEAR, 0.0)
    gs.z_faces = ctypes.cast(zf, ctypes.POINTER(ctypes.c_double))
    assert lib.oc_grid_create(ctypes.byref(gs), ctypes.byref(g)) == 0
    assert lib.oc_model_workspace_size(g, ctypes.byref(md), ctypes.byref(n)) == -5
    assert lib.oc_grid_destroy(g) == 0
    assert lib.oc_set_immersed(None, None, None) == -1
    assert lib.oc_pressure_stats(None, None, None, None) == -1


def test_new_calls_reject_null_arguments():
    lib = oc.load_library()
    assert lib.oc_sync_check(None, None) == -1
    assert lib.oc_autotune(None, None) == -1
    assert lib.oc_ensemble_set_tuning(None, None) == -1
    assert lib.oc_diagnostics(None, None, None) == -1
