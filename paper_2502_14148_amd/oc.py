"""Thin ctypes binding of liboc.so (the C ABI in include/oc.h).

Argument marshalling only: every step of the model runs in the HIP kernels
of the library.  Device memory and streams come from PyTorch: the model's
workspace is a torch uint8 tensor on the GPU and calls are enqueued on the
current torch stream.  Loading fails loudly if the library is missing.
"""
import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liboc.so")

OC_OK = 0
OC_ERR = {-1: "OC_ERR_ARG", -2: "OC_ERR_SHAPE", -3: "OC_ERR_DTYPE", -4: "OC_ERR_DEVICE",
          -5: "OC_ERR_UNSUPPORTED", -6: "OC_ERR_NONFINITE"}
OC_PERIODIC, OC_BOUNDED = 0, 1
OC_RECTILINEAR, OC_LATLON = 0, 1
OC_NONHYDROSTATIC, OC_HYDROSTATIC = 0, 1
BARO_FIELDS = {"eta": 16, "U": 17, "V": 18, "GU": 19, "GV": 20, "tau_x": 21, "tau_y": 22}
OC_FP64, OC_FP32_MIXED = 0, 1
ADVECTION = {"none": 0, "weno5z": 1, "weno5_linear": 2, "weno7z": 3, "weno7_linear": 4,
             "weno9z": 5, "weno9_linear": 6}
OC_F32, OC_F64 = 0, 1
OC_MAX_TRACERS = 4
OC_NDIAG = 12

EXPORTS = ("oc_last_error", "oc_grid_create", "oc_grid_destroy", "oc_model_workspace_size",
           "oc_model_create", "oc_model_destroy", "oc_set_state", "oc_get_state",
           "oc_tendencies", "oc_get_tendency", "oc_pressure_solve", "oc_get_pressure",
           "oc_rk3_step", "oc_diagnostics", "oc_profile", "oc_profile_read", "oc_profile_classes",
           "oc_free_surface_substeps", "oc_hydrostatic_step", "oc_mlp_workspace_size",
           "oc_mlp_create",
           "oc_mlp_destroy", "oc_mlp_set_params", "oc_mlp_get_params", "oc_mlp_forward",
           "oc_mlp_gradients", "oc_mlp_train_step", "oc_model_set_closure",
           "oc_ensemble_workspace_size", "oc_ensemble_create", "oc_ensemble_step",
           "oc_ensemble_tuning", "oc_ensemble_destroy", "oc_closure_features",
           "oc_coarse_grain", "oc_implicit_vertical_diffusion", "oc_set_immersed",
           "oc_pressure_stats", "oc_sync_check", "oc_autotune", "oc_ensemble_set_tuning",
           "oc_diagnostics_noalloc")
OC_ENS_TUNE, OC_ENS_GRAPH = 1, 2
ENS_TILES = ("32x8", "16x8", "8x8")
OC_MLP_NPARAM = 195076
MLP_SHAPES = (("W1", (256, 500)), ("b1", (256,)), ("W2", (256, 256)), ("b2", (256,)),
              ("W3", (4, 256)), ("b3", (4,)))
OC_NPROF = 15
PROF_CLASSES = ("tendency", "fft_x_fwd", "fft_y_fwd", "z_solve", "fft_y_inv", "fft_x_inv",
                "project", "halo", "closure", "hydro_diag", "hydro_tendency", "barotropic",
                "implicit_z", "les", "cg")
LES = {"none": 0, "smagorinsky": 1, "amd": 2}


class GridDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("topology_z", ctypes.c_int32),
                ("x0", ctypes.c_double), ("lx", ctypes.c_double),
                ("y0", ctypes.c_double), ("ly", ctypes.c_double),
                ("z0", ctypes.c_double), ("lz", ctypes.c_double),
                ("coord", ctypes.c_int32), ("radius", ctypes.c_double),
                ("z_faces", ctypes.POINTER(ctypes.c_double))]


class ModelDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("advection", ctypes.c_int32),
                ("weno_eps", ctypes.c_double), ("weno_q", ctypes.c_int32),
                ("ntracers", ctypes.c_int32), ("buoyancy", ctypes.c_int32),
                ("f", ctypes.c_double), ("g", ctypes.c_double), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("t_ref", ctypes.c_double), ("s_ref", ctypes.c_double),
                ("nu", ctypes.c_double), ("kappa", ctypes.c_double),
                ("top_flux", ctypes.c_double * OC_MAX_TRACERS),
                ("depth", ctypes.c_double), ("omega", ctypes.c_double),
                ("closure", ctypes.c_int32), ("implicit_z", ctypes.c_int32),
                ("les", ctypes.c_int32), ("les_c", ctypes.c_double), ("les_cb", ctypes.c_double),
                ("les_pr", ctypes.c_double), ("immersed", ctypes.c_int32),
                ("cg_tol", ctypes.c_double), ("cg_maxiter", ctypes.c_int32)]


class OcError(RuntimeError):
    pass


_lib = None


def load_library(path=_LIB_PATH):
    """Load liboc.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OcError(f"{path} is missing: build it with `python -m paper_2502_14148_amd.build`")
    # PyTorch ships its own HIP runtime under the same soname: it must be the
    # one loaded, or device memory from torch is foreign to the library
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i32, i64p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
    lib.oc_last_error.restype = ctypes.c_char_p
    lib.oc_last_error.argtypes = []
    sig = {
        "oc_grid_create": [ctypes.POINTER(GridDesc), ctypes.POINTER(vp)],
        "oc_grid_destroy": [vp],
        "oc_model_workspace_size": [vp, ctypes.POINTER(ModelDesc), ctypes.POINTER(ctypes.c_uint64)],
        "oc_model_create": [vp, ctypes.POINTER(ModelDesc), vp, ctypes.c_uint64, ctypes.POINTER(vp)],
        "oc_model_destroy": [vp],
        "oc_set_state": [vp, i32, vp, i32, i32, i64p, vp],
        "oc_get_state": [vp, i32, vp, i32, i32, i64p, vp],
        "oc_tendencies": [vp, vp],
        "oc_get_tendency": [vp, i32, vp, i32, i32, i64p, vp],
        "oc_pressure_solve": [vp, ctypes.c_double, vp],
        "oc_get_pressure": [vp, vp, i32, vp],
        "oc_rk3_step": [vp, ctypes.c_double, i32, vp],
        "oc_diagnostics": [vp, ctypes.POINTER(ctypes.c_double), vp],
        "oc_profile": [vp, i32],
        "oc_profile_classes": [vp, ctypes.c_uint32],
        "oc_profile_read": [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)],
        "oc_free_surface_substeps": [vp, ctypes.c_double, i32, i32, ctypes.POINTER(ctypes.c_double), vp],
        "oc_hydrostatic_step": [vp, ctypes.c_double, i32, i32, ctypes.POINTER(ctypes.c_double), i32,
                                vp],
        "oc_mlp_workspace_size": [i32, ctypes.POINTER(ctypes.c_uint64)],
        "oc_mlp_create": [i32, vp, ctypes.c_uint64, ctypes.POINTER(vp)],
        "oc_mlp_destroy": [vp],
        "oc_mlp_set_params": [vp, vp, vp],
        "oc_mlp_get_params": [vp, vp, vp],
        "oc_mlp_forward": [vp, vp, i32, vp, vp],
        "oc_mlp_gradients": [vp, vp, vp, i32, vp, ctypes.POINTER(ctypes.c_double), vp],
        "oc_mlp_train_step": [vp, vp, vp, i32, ctypes.c_float, ctypes.POINTER(ctypes.c_double), vp],
        "oc_model_set_closure": [vp, vp, ctypes.POINTER(ctypes.c_double), vp],
        "oc_ensemble_workspace_size": [ctypes.POINTER(vp), i32, ctypes.POINTER(ctypes.c_uint64)],
        "oc_ensemble_create": [ctypes.POINTER(vp), i32, vp, ctypes.c_uint64, i32,
                               ctypes.POINTER(vp)],
        "oc_ensemble_step": [vp, ctypes.c_double, i32, vp],
        "oc_ensemble_tuning": [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)],
        "oc_ensemble_destroy": [vp],
        "oc_closure_features": [vp, ctypes.POINTER(ctypes.c_double), vp, vp],
        "oc_coarse_grain": [vp, vp, vp, vp],
        "oc_implicit_vertical_diffusion": [vp, ctypes.c_double, vp],
        "oc_set_immersed": [vp, vp, vp],
        "oc_pressure_stats": [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                              vp],
        "oc_sync_check": [vp, vp],
        "oc_diagnostics_noalloc": [vp, vp, vp],
        "oc_autotune": [vp, ctypes.c_char_p],
        "oc_ensemble_set_tuning": [vp, ctypes.POINTER(ctypes.c_int32)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != OC_OK:
        msg = _lib.oc_last_error().decode()
        raise OcError(f"{OC_ERR.get(rc, rc)}: {msg}")


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Model:
    """A model on the GPU, configured from a Physics record (nonhydrostatic)
    or a HydrostaticPhysics record (hydrostatic, lat-lon), see
    paper_2502_14148_amd.inputs."""

    def __init__(self, ph, precision="fp64", device="cuda:0"):
        import torch
        lib = load_library()
        self.ph = ph
        self.device = torch.device(device)
        self.precision = precision
        self.hydrostatic = getattr(ph, "kind", "nonhydrostatic") == "hydrostatic"
        self.fields = ("u", "v", "w") + tuple(ph.tracers)
        md = ModelDesc()
        if self.hydrostatic:
            gd = GridDesc(ph.nx, ph.ny, ph.nz, OC_BOUNDED, ph.lon0, ph.lon_extent, ph.lat0,
                          ph.lat_extent, -ph.depth, ph.depth, OC_LATLON, ph.radius)
            md.kind, md.depth, md.omega = OC_HYDROSTATIC, ph.depth, ph.omega
            md.f = 0.0
        else:
            gd = GridDesc(ph.nx, ph.ny, ph.nz, OC_BOUNDED if ph.z_bounded else OC_PERIODIC,
                          ph.x0, ph.lx, ph.y0, ph.ly, ph.z0, ph.lz, OC_RECTILINEAR, 0.0)
            zf = getattr(ph, "z_faces", None)
            if zf is not None:
                # copied by oc_grid_create
                self._zf = (ctypes.c_double * len(zf))(*[float(z) for z in zf])
                gd.z_faces = ctypes.cast(self._zf, ctypes.POINTER(ctypes.c_double))
            md.kind = OC_NONHYDROSTATIC
            md.f = ph.f
            md.implicit_z = 1 if getattr(ph, "implicit_z", False) else 0
            md.les = LES[getattr(ph, "les", "none")]
            if md.les == LES["smagorinsky"]:
                md.les_c, md.les_cb, md.les_pr = ph.les_cs, ph.les_cb, ph.les_pr
            elif md.les == LES["amd"]:
                md.les_c, md.les_cb, md.les_pr = ph.les_camd, 0.0, 1.0
            solid = getattr(ph, "solid", None)
            if solid is not None:
                md.immersed = 1
                md.cg_tol = getattr(ph, "cg_tol", 1e-13)
                md.cg_maxiter = getattr(ph, "cg_maxiter", 200)
        md.precision = OC_FP64 if precision == "fp64" else OC_FP32_MIXED
        md.advection = ADVECTION[ph.advection]
        md.weno_eps = ph.weno_eps
        md.weno_q = ph.weno_q
        md.ntracers = len(ph.tracers)
        md.buoyancy = 1 if ph.buoyancy else 0
        md.closure = 1 if getattr(ph, "closure", False) else 0
        md.g, md.alpha, md.beta = ph.g, ph.alpha, ph.beta
        md.t_ref, md.s_ref = ph.t_ref, ph.s_ref
        md.nu, md.kappa = ph.nu, ph.kappa
        top = getattr(ph, "top_flux", {})
        for q, name in enumerate(ph.tracers):
            md.top_flux[q] = top.get(name, 0.0)
        self._gd, self._md = gd, md
        self._grid = ctypes.c_void_p()
        _check(lib.oc_grid_create(ctypes.byref(gd), ctypes.byref(self._grid)))
        nbytes = ctypes.c_uint64()
        _check(lib.oc_model_workspace_size(self._grid, ctypes.byref(md), ctypes.byref(nbytes)))
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
            self._model = ctypes.c_void_p()
            _check(lib.oc_model_create(self._grid, ctypes.byref(md),
                                       ctypes.c_void_p(self.workspace.data_ptr()),
                                       ctypes.c_uint64(nbytes.value), ctypes.byref(self._model)))
        if md.immersed:
            self.set_immersed(ph.solid)

    def __del__(self):
        try:
            if getattr(self, "_model", None):
                _lib.oc_model_destroy(self._model)
            if getattr(self, "_grid", None):
                _lib.oc_grid_destroy(self._grid)
        except Exception:
            pass

    # -- helpers -----------------------------------------------------------
    def field_id(self, name):
        if name in BARO_FIELDS:
            return BARO_FIELDS[name]
        return self.fields.index(name)

    def shape_of(self, name):
        ph = self.ph
        if name in BARO_FIELDS:
            return (1, ph.ny + (1 if name in ("V", "GV", "tau_y") else 0), ph.nx)
        zb = True if self.hydrostatic else ph.z_bounded
        nzf = ph.nz + 1 if (name == "w" and zb) else ph.nz
        nyf = ph.ny + 1 if (name == "v" and self.hydrostatic) else ph.ny
        return (nzf, nyf, ph.nx)

    def _io(self, fn, name, buf):
        """Call a set/get entry point with a numpy (host) or torch array."""
        import torch
        shape = (ctypes.c_int64 * 3)(*buf.shape)
        if isinstance(buf, torch.Tensor):
            assert buf.is_contiguous()
            dtype = OC_F64 if buf.dtype == torch.float64 else OC_F32
            ptr, on_dev = buf.data_ptr(), 1 if buf.is_cuda else 0
        else:
            assert buf.flags["C_CONTIGUOUS"]
            dtype = OC_F64 if buf.dtype == np.float64 else OC_F32
            ptr, on_dev = buf.ctypes.data, 0
        _check(fn(self._model, self.field_id(name), ctypes.c_void_p(ptr), dtype, on_dev, shape,
                  _stream()))

    # -- C ABI -------------------------------------------------------------
    def set_state(self, name, arr):
        self._io(_lib.oc_set_state, name, arr)

    def set_states(self, d):
        """Set every prognostic field present in d (w of the hydrostatic model
        is diagnostic and skipped)."""
        for name in self.fields:
            if self.hydrostatic and name == "w":
                continue
            if name in d:
                self.set_state(name, d[name])

    def get_state(self, name, out=None, dtype=np.float64):
        if out is None:
            out = np.empty(self.shape_of(name), dtype=dtype)
        self._io(_lib.oc_get_state, name, out)
        return out

    def get_states(self):
        return {n: self.get_state(n) for n in self.fields}

    def tendencies(self):
        _check(_lib.oc_tendencies(self._model, _stream()))

    def get_tendency(self, name, out=None, dtype=np.float64):
        if out is None:
            out = np.empty(self.shape_of(name), dtype=dtype)
        self._io(_lib.oc_get_tendency, name, out)
        return out

    def pressure_solve(self, dt_eff):
        _check(_lib.oc_pressure_solve(self._model, ctypes.c_double(dt_eff), _stream()))

    def get_pressure(self, out=None):
        if out is None:
            out = np.empty((self.ph.nz, self.ph.ny, self.ph.nx), dtype=np.float64)
        import torch
        if isinstance(out, torch.Tensor):
            _check(_lib.oc_get_pressure(self._model, ctypes.c_void_p(out.data_ptr()), 1, _stream()))
        else:
            _check(_lib.oc_get_pressure(self._model, ctypes.c_void_p(out.ctypes.data), 0, _stream()))
        return out

    def rk3_step(self, dt, nsteps=1):
        _check(_lib.oc_rk3_step(self._model, ctypes.c_double(dt), ctypes.c_int32(nsteps), _stream()))

    def set_immersed(self, solid):
        """Immersed cells ((nz, ny, nx) booleans, True = immersed)."""
        a = np.ascontiguousarray(np.asarray(solid, dtype=np.uint8))
        assert a.shape == (self.ph.nz, self.ph.ny, self.ph.nx)
        _check(_lib.oc_set_immersed(self._model, ctypes.c_void_p(a.ctypes.data), _stream()))

    def pressure_stats(self):
        """(iterations, relative residual) of the last immersed pressure solve."""
        it = ctypes.c_int32()
        res = ctypes.c_double()
        _check(_lib.oc_pressure_stats(self._model, ctypes.byref(it), ctypes.byref(res), _stream()))
        return it.value, res.value

    def implicit_vertical_diffusion(self, dt_eff):
        _check(_lib.oc_implicit_vertical_diffusion(self._model, ctypes.c_double(dt_eff), _stream()))

    def diagnostics(self):
        out = (ctypes.c_double * OC_NDIAG)()
        _check(_lib.oc_diagnostics(self._model, out, _stream()))
        return {"div_scaled_by_dx": out[0], "max_u": out[1], "max_v": out[2], "max_w": out[3],
                "tracer_integrals": list(out[4:4 + len(self.ph.tracers)]),
                "momentum": (out[8], out[9], out[10]), "cfl_rate": out[11]}

    def diagnostics_noalloc(self, out):
        """Enqueue the diagnostics into `out` (FP64 device tensor of
        OC_NDIAG + 1 values: the oc_diagnostics values, then the count of
        non-finite state values); no allocation, no synchronisation."""
        assert out.is_cuda and out.dtype.is_floating_point and out.element_size() == 8
        assert out.is_contiguous() and out.numel() >= OC_NDIAG + 1
        _check(_lib.oc_diagnostics_noalloc(self._model, ctypes.c_void_p(out.data_ptr()),
                                           _stream()))
        return out

    def sync_check(self):
        """Synchronise the current stream; raises on a device error or a
        non-finite state (OC_ERR_NONFINITE)."""
        _check(_lib.oc_sync_check(self._model, _stream()))

    def profile(self, enable=True, classes=None):
        """Start (clearing the totals) or stop event timing; `classes` (names
        from PROF_CLASSES) restricts the recording to those kernel classes,
        None records all of them."""
        if enable:
            mask = (1 << len(PROF_CLASSES)) - 1 if classes is None else \
                sum(1 << PROF_CLASSES.index(c) for c in set(classes))
            _check(_lib.oc_profile_classes(self._model, mask))
        _check(_lib.oc_profile(self._model, 1 if enable else 0))

    def profile_read(self):
        ms = (ctypes.c_double * OC_NPROF)()
        n = (ctypes.c_int64 * OC_NPROF)()
        _check(_lib.oc_profile_read(self._model, ms, n))
        return {c: (ms[i], n[i]) for i, c in enumerate(PROF_CLASSES)}

    def set_closure(self, net, stats=None):
        """Attach a trained Mlp (stats: 16 numbers, input mean/std of u, v, w, b
        and output mean/std of the 4 fluxes) or detach it (net=None)."""
        if net is None:
            _check(_lib.oc_model_set_closure(self._model, None, None, _stream()))
            self._net = None
            return
        st = np.ascontiguousarray(stats, dtype=np.float64)
        assert st.size == 16
        _check(_lib.oc_model_set_closure(self._model, net._h,
                                         st.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         _stream()))
        self._net = net   # the network must outlive the attachment

    def closure_features(self, stats, out=None):
        """FP32 device tensor (ncell, 500) of standardised network inputs of
        the current state; stats: 16 numbers (the first 8 are used)."""
        import torch
        n = self.ph.nx * self.ph.ny * self.ph.nz
        if out is None:
            out = torch.empty((n, 500), dtype=torch.float32, device=self.device)
        st = np.ascontiguousarray(stats, dtype=np.float64)
        _check(_lib.oc_closure_features(self._model,
                                        st.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    def coarse_grain_from(self, fine, fluxes=None):
        """This model's state becomes the coarse-grained state of `fine`;
        fluxes (FP32 device tensor (4, nz, ny, nx) of this grid, optional)
        receives the vertical subgrid fluxes."""
        ptr = ctypes.c_void_p(fluxes.data_ptr()) if fluxes is not None else None
        _check(_lib.oc_coarse_grain(fine._model, self._model, ptr, _stream()))
        return fluxes

    def free_surface_substeps(self, dt, N, weights):
        w = np.ascontiguousarray(weights, dtype=np.float64)
        _check(_lib.oc_free_surface_substeps(self._model, ctypes.c_double(dt), ctypes.c_int32(N),
                                             ctypes.c_int32(len(w)),
                                             w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             _stream()))

    def hydrostatic_step(self, dt, N, weights, nsteps=1):
        w = np.ascontiguousarray(weights, dtype=np.float64)
        _check(_lib.oc_hydrostatic_step(self._model, ctypes.c_double(dt), ctypes.c_int32(N),
                                        ctypes.c_int32(len(w)),
                                        w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        ctypes.c_int32(nsteps), _stream()))


def pack_mlp(params):
    """Dict of arrays (W1, b1, W2, b2, W3, b3) -> packed FP32 vector."""
    return np.concatenate([np.asarray(params[k], dtype=np.float32).ravel() for k, _ in MLP_SHAPES])


def unpack_mlp(vec):
    out, o = {}, 0
    for k, shp in MLP_SHAPES:
        n = int(np.prod(shp))
        out[k] = np.asarray(vec[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


class Mlp:
    """The MLP closure network on the GPU (BF16 MFMA, FP32 master weights)."""

    def __init__(self, max_batch, device="cuda:0"):
        import torch
        lib = load_library()
        self.device = torch.device(device)
        nbytes = ctypes.c_uint64()
        _check(lib.oc_mlp_workspace_size(max_batch, ctypes.byref(nbytes)))
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
            self._h = ctypes.c_void_p()
            _check(lib.oc_mlp_create(max_batch, ctypes.c_void_p(self.workspace.data_ptr()),
                                     ctypes.c_uint64(nbytes.value), ctypes.byref(self._h)))
        self.max_batch = max_batch

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                _lib.oc_mlp_destroy(self._h)
        except Exception:
            pass

    def set_params(self, params):
        v = np.ascontiguousarray(pack_mlp(params) if isinstance(params, dict) else params,
                                 dtype=np.float32)
        assert v.size == OC_MLP_NPARAM
        _check(_lib.oc_mlp_set_params(self._h, ctypes.c_void_p(v.ctypes.data), _stream()))

    def get_params(self):
        v = np.empty(OC_MLP_NPARAM, dtype=np.float32)
        _check(_lib.oc_mlp_get_params(self._h, ctypes.c_void_p(v.ctypes.data), _stream()))
        return unpack_mlp(v)

    def forward(self, x):
        import torch
        x = x.contiguous()
        y = torch.empty((x.shape[0], 4), dtype=torch.float32, device=x.device)
        _check(_lib.oc_mlp_forward(self._h, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                   ctypes.c_void_p(y.data_ptr()), _stream()))
        return y

    def gradients(self, x, t):
        import torch
        g = torch.empty(OC_MLP_NPARAM, dtype=torch.float32, device=x.device)
        loss = ctypes.c_double()
        _check(_lib.oc_mlp_gradients(self._h, ctypes.c_void_p(x.contiguous().data_ptr()),
                                     ctypes.c_void_p(t.contiguous().data_ptr()), x.shape[0],
                                     ctypes.c_void_p(g.data_ptr()), ctypes.byref(loss), _stream()))
        return g, loss.value

    def train_step(self, x, t, lr, want_loss=True):
        loss = ctypes.c_double()
        _check(_lib.oc_mlp_train_step(self._h, ctypes.c_void_p(x.contiguous().data_ptr()),
                                      ctypes.c_void_p(t.contiguous().data_ptr()), x.shape[0],
                                      ctypes.c_float(lr),
                                      ctypes.byref(loss) if want_loss else None, _stream()))
        return loss.value if want_loss else None


class Ensemble:
    """Many Model instances stepped together (one fused tendency launch per
    substage over all members, batched Poisson passes, optional HIP graph
    replay and autotuned launch configuration)."""

    def __init__(self, models, tune=False, graph=False, device="cuda:0"):
        import torch
        lib = load_library()
        self.models = list(models)           # kept alive: the ensemble borrows them
        n = len(self.models)
        arr = (ctypes.c_void_p * n)(*[m._model.value for m in self.models])
        nbytes = ctypes.c_uint64()
        _check(lib.oc_ensemble_workspace_size(arr, n, ctypes.byref(nbytes)))
        flags = (OC_ENS_TUNE if tune else 0) | (OC_ENS_GRAPH if graph else 0)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=device)
        self._h = ctypes.c_void_p()
        _check(lib.oc_ensemble_create(arr, n, ctypes.c_void_p(self.workspace.data_ptr()),
                                      ctypes.c_uint64(nbytes.value), flags, ctypes.byref(self._h)))

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                _lib.oc_ensemble_destroy(self._h)
        except Exception:
            pass

    def step(self, dt, nsteps=1):
        _check(_lib.oc_ensemble_step(self._h, ctypes.c_double(dt), ctypes.c_int32(nsteps),
                                     _stream()))

    def tuning(self):
        out = (ctypes.c_int32 * 6)()
        ms = ctypes.c_double()
        _check(_lib.oc_ensemble_tuning(self._h, out, ctypes.byref(ms)))
        return {"tile": ENS_TILES[out[0]], "persistent": bool(out[1]),
                "nblocks": out[2], "kc_div": out[3],
                "source": ("default", "timed", "cache", "set")[out[4]], "items": out[5],
                "ms": ms.value}

    def autotune(self, cache_path=None):
        """Time the launch configurations (or read the choice from the
        JSON-lines cache file) and keep the fastest."""
        p = None if cache_path is None else os.fsencode(str(cache_path))
        _check(_lib.oc_autotune(self._h, p))
        return self.tuning()

    def set_tuning(self, tile="32x8", persistent=False, kc_div=1024):
        t = (ctypes.c_int32 * 3)(ENS_TILES.index(tile), 1 if persistent else 0, kc_div)
        _check(_lib.oc_ensemble_set_tuning(self._h, t))
        return self.tuning()
