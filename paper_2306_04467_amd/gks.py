"""Thin ctypes binding of the HIP library's C ABI (include/gks.h).

Argument marshalling only: every step of the scheme runs in the library's kernels.  The binding
raises if the shared object is missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import json
import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GKS_LIBRARY may name another build of the same ABI (used to compare kernel variants)
LIB_PATH = os.environ.get("GKS_LIBRARY", os.path.join(_HERE, "libgks.so"))
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p
_fp = ctypes.POINTER(ctypes.c_float)
_u8p = ctypes.POINTER(ctypes.c_uint8)

GKS_OK, GKS_EINVAL, GKS_ENOMEM, GKS_EDEVICE, GKS_EMESH, GKS_ENONFINITE, GKS_EUNSUPPORTED = range(7)
GKS_BC_WALL, GKS_BC_PERIODIC, GKS_BC_FREE = 0, 1, 2
BOUNDARIES = {"wall": GKS_BC_WALL, "periodic": GKS_BC_PERIODIC, "free": GKS_BC_FREE}
GKS_FP64, GKS_FP32_MIXED = 0, 1
PRECISIONS = {"fp64": GKS_FP64, "fp32": GKS_FP32_MIXED}

# every entry point declared in include/gks.h
SYMBOLS = ("gks_mesh_create", "gks_mesh_batch", "gks_mesh_destroy", "gks_mesh_info", "gks_mesh_scenario",
           "gks_state_init", "gks_state_destroy", "gks_stage", "gks_step", "gks_batch_step", "gks_state_read",
           "gks_state_time", "gks_state_mass", "gks_state_mass_noalloc", "gks_state_diagnostics", "gks_state_check",
           "gks_state_checkpoint_size", "gks_state_save", "gks_state_load", "gks_state_buffer", "gks_profile", "gks_profile_read",
           "gks_indicator_set", "gks_indicator_eval", "gks_state_features", "gks_state_labels",
           "gks_trainer_create", "gks_trainer_destroy", "gks_trainer_add", "gks_trainer_add_state",
           "gks_trainer_info", "gks_trainer_grad", "gks_trainer_fit", "gks_trainer_params", "gks_trainer_logits",
           "gks_trainer_threshold", "gks_autotune", "gks_debug_bounds", "gks_last_error")
_VOID = ("gks_mesh_destroy", "gks_state_destroy", "gks_trainer_destroy", "gks_last_error")
MLP_PARAMS, MLP_FEATURES = 7105, 44
BUFFERS = {"rech": (0, 12, True), "recm": (1, 96, False), "r0": (2, 2, False), "eoh": (3, 6, True),
           "eom": (4, 24, False), "skip": (5, 1, None), "src": (6, 8, False)}
KERNELS = ("ghost", "recon", "hhat", "plane", "flux", "update", "dt", "indicator")


class GksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gks error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("G", ctypes.c_double), ("chi", ctypes.c_double), ("cfl", ctypes.c_double),
                ("eps", ctypes.c_double), ("eps_num", ctypes.c_double), ("t_end", ctypes.c_double),
                ("precision", ctypes.c_int32), ("linear", ctypes.c_int32), ("alpha_mode", ctypes.c_int32),
                ("src_order", ctypes.c_int32), ("grad_mode", ctypes.c_int32),
                ("h_dry", ctypes.c_double)]


ALPHA_MODES = {"reading": 0, "paper": 1}
SRC_ORDERS = (2, 4)
GRAD_MODES = {"continuous": 0, "discontinuous": 1}


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run python paper_2306_04467_amd/build.py)")
    # stream handles come from torch: load torch's HIP runtime first so that the library binds to
    # the same one
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    lib.gks_last_error.restype = ctypes.c_char_p
    lib.gks_mesh_create.argtypes = [_dp, ctypes.c_int64, _i32p, ctypes.c_int64, _dp, ctypes.c_int32, _dp,
                                    ctypes.POINTER(_vp)]
    lib.gks_mesh_batch.argtypes = [ctypes.POINTER(_vp), ctypes.c_int32, ctypes.POINTER(_vp)]
    lib.gks_mesh_destroy.argtypes = [_vp]
    lib.gks_mesh_destroy.restype = None
    lib.gks_mesh_info.argtypes = [_vp, _i64p, _i64p, _i64p, _i32p]
    lib.gks_mesh_scenario.argtypes = [_vp, ctypes.c_int32, _i64p, _i64p]
    lib.gks_state_init.argtypes = [_vp, ctypes.POINTER(Params), _dp, _dp, _vp, ctypes.POINTER(_vp)]
    lib.gks_state_destroy.argtypes = [_vp]
    lib.gks_state_destroy.restype = None
    lib.gks_stage.argtypes = [_vp, ctypes.c_int32, _dp]
    lib.gks_step.argtypes = [_vp, ctypes.c_int32, _dp]
    lib.gks_batch_step.argtypes = [_vp, ctypes.c_int32]
    lib.gks_state_read.argtypes = [_vp, _dp, _dp, _dp]
    lib.gks_state_time.argtypes = [_vp, ctypes.c_int32, _dp, _dp]
    lib.gks_state_mass.argtypes = [_vp, ctypes.c_int32, _dp]
    lib.gks_state_mass_noalloc.argtypes = [_vp, ctypes.c_int32, _dp]
    lib.gks_state_diagnostics.argtypes = [_vp, ctypes.c_int32, _dp]
    lib.gks_state_check.argtypes = [_vp, _i64p]
    lib.gks_debug_bounds.argtypes = [ctypes.c_int32, _i32p]
    lib.gks_state_checkpoint_size.argtypes = [_vp, _i64p]
    lib.gks_state_save.argtypes = [_vp, _vp, ctypes.c_int64]
    lib.gks_state_load.argtypes = [_vp, _vp, ctypes.c_int64]
    lib.gks_state_buffer.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int64]
    lib.gks_profile.argtypes = [_vp, ctypes.c_int32]
    lib.gks_profile_read.argtypes = [_vp, ctypes.c_int32, _dp, _i64p]
    lib.gks_indicator_set.argtypes = [_vp, _fp, ctypes.c_float]
    lib.gks_indicator_eval.argtypes = [_vp, _fp, _u8p, _i64p]
    lib.gks_state_features.argtypes = [_vp, _fp]
    lib.gks_state_labels.argtypes = [_vp, ctypes.c_double, _u8p]
    lib.gks_trainer_create.argtypes = [ctypes.c_int64, ctypes.c_int32, _fp, _vp, ctypes.POINTER(_vp)]
    lib.gks_trainer_destroy.argtypes = [_vp]
    lib.gks_trainer_destroy.restype = None
    lib.gks_trainer_add.argtypes = [_vp, _fp, _u8p, ctypes.c_int64]
    lib.gks_trainer_add_state.argtypes = [_vp, _vp, ctypes.c_double, _i64p]
    lib.gks_trainer_info.argtypes = [_vp, _i64p, _i64p]
    lib.gks_trainer_grad.argtypes = [_vp, _i32p, ctypes.c_int32, _fp, _fp]
    lib.gks_trainer_fit.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_uint64, _fp]
    lib.gks_trainer_params.argtypes = [_vp, _fp]
    lib.gks_trainer_logits.argtypes = [_vp, _fp]
    lib.gks_trainer_threshold.argtypes = [_vp, ctypes.c_double, _fp]
    lib.gks_autotune.argtypes = [_vp, ctypes.c_int32, _i32p]
    for name in SYMBOLS:
        if name not in _VOID:
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def debug_bounds(reset=False):
    """Index checks of the checked build (see gks_debug_bounds): 1 after an out-of-range index,
    else 0; raises GksError(GKS_EUNSUPPORTED) in the ordinary build."""
    v = ctypes.c_int32()
    _check(load().gks_debug_bounds(int(bool(reset)), ctypes.byref(v)))
    return v.value


def _check(code):
    if code != GKS_OK:
        raise GksError(code, load().gks_last_error().decode())


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _pf(a):
    return a.ctypes.data_as(_fp)


def _pu8(a):
    return a.ctypes.data_as(_u8p)


def current_stream():
    """Handle of torch's current HIP stream (device memory and streams come from PyTorch)."""
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible to torch")
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Mesh:
    def __init__(self, node_xy=None, tri=None, node_B=None, periodic_L=None, _handle=None, boundary=None):
        lib = load()
        if _handle is None:
            self.node_xy = _f64(node_xy)
            self.tri = np.ascontiguousarray(tri, dtype=np.int32)
            nB = None if node_B is None else _f64(node_B)
            per = None if periodic_L is None else _f64(periodic_L)
            if boundary is None:
                boundary = "periodic" if per is not None else "wall"
            h = _vp()
            _check(lib.gks_mesh_create(_d(self.node_xy), self.node_xy.shape[0], self.tri.ctypes.data_as(_i32p),
                                       self.tri.shape[0], None if nB is None else _d(nB), BOUNDARIES[boundary],
                                       None if per is None else _d(per), ctypes.byref(h)))
            _handle = h
        self._h = _handle
        T, E, NG, S = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check(lib.gks_mesh_info(self._h, ctypes.byref(T), ctypes.byref(E), ctypes.byref(NG), ctypes.byref(S)))
        self.n_tri, self.n_edges, self.n_ghost, self.n_scenarios = T.value, E.value, NG.value, S.value

    @classmethod
    def from_scenario(cls, sc):
        return cls(sc.node_xy, sc.tri, sc.node_B, sc.periodic_L if sc.boundary == "periodic" else None,
                   boundary=sc.boundary)

    @classmethod
    def batch(cls, meshes):
        """Concatenate single meshes into one batch mesh (the inputs stay usable)."""
        arr = (_vp * len(meshes))(*[m._h for m in meshes])
        h = _vp()
        _check(load().gks_mesh_batch(arr, len(meshes), ctypes.byref(h)))
        return cls(_handle=h)

    def scenario_range(self, s):
        a, n = ctypes.c_int64(), ctypes.c_int64()
        _check(load().gks_mesh_scenario(self._h, int(s), ctypes.byref(a), ctypes.byref(n)))
        return a.value, n.value

    def close(self):
        if getattr(self, "_h", None):
            load().gks_mesh_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit the module's globals may already be gone; the process's end frees
        # the device memory then
        if not _finalizing():
            self.close()


def make_params(G=9.81, chi=0.98, cfl=0.3, eps=0.05, eps_num=5.0, t_end=0.0, precision="fp64", linear=False,
                alpha_mode="reading", src_order=2, grad_mode="continuous", h_dry=0.0):
    return Params(G, chi, cfl, eps, eps_num, t_end, PRECISIONS[precision], int(linear), ALPHA_MODES[alpha_mode],
                  int(src_order), GRAD_MODES[grad_mode], float(h_dry))


class State:
    """State on a (single or batch) mesh.  params: one Params, or a list with one per scenario."""

    def __init__(self, mesh: Mesh, W0, gradW0, params=None, stream=None, **kw):
        lib = load()
        self.mesh = mesh
        T = mesh.n_tri
        W0 = _f64(W0).reshape(6, T)
        gW0 = _f64(gradW0).reshape(6, 2, T)
        if params is None:
            params = make_params(**kw)
        plist = list(params) if isinstance(params, (list, tuple)) else [params]
        if len(plist) != mesh.n_scenarios:
            raise ValueError("one Params per scenario is needed")
        self._params = (Params * len(plist))(*plist)
        if stream is None:
            stream = current_stream()
        self.stream = stream
        h = _vp()
        _check(lib.gks_state_init(mesh._h, self._params, _d(W0), _d(gW0), stream, ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_scenario(cls, mesh, sc, precision="fp64", linear=False, t_end=0.0, alpha_mode="reading",
                      src_order=2, grad_mode="continuous", h_dry=None, **kw):
        """h_dry: the wet/dry threshold, by default the scenario's own (0 where it has none)."""
        if h_dry is None:
            h_dry = getattr(sc, "h_dry", 0.0)
        p = make_params(G=sc.G, chi=sc.chi, cfl=sc.cfl, t_end=t_end, precision=precision, linear=linear,
                        alpha_mode=alpha_mode, src_order=src_order, grad_mode=grad_mode, h_dry=h_dry)
        return cls(mesh, sc.W0, sc.gradW0, params=p, **kw)

    @classmethod
    def from_scenarios(cls, batch_mesh, scs, precision="fp64", linear=False, src_order=2, grad_mode="continuous",
                       **kw):
        ps = [make_params(G=s.G, chi=s.chi, cfl=s.cfl, t_end=s.t_end if s.t_end < 1e8 else 0.0,
                          precision=precision, linear=linear, src_order=src_order, grad_mode=grad_mode,
                          h_dry=getattr(s, "h_dry", 0.0))
              for s in scs]
        W0 = np.concatenate([s.W0 for s in scs], axis=1)
        gW0 = np.concatenate([s.gradW0 for s in scs], axis=2)
        return cls(batch_mesh, W0, gW0, params=ps, **kw)

    def stage(self, k, dt=None):
        d = None if dt is None else ctypes.byref(ctypes.c_double(dt))
        _check(load().gks_stage(self._h, int(k), d))

    def step(self, n=1, want_dt=False):
        if want_dt:
            d = ctypes.c_double()
            _check(load().gks_step(self._h, int(n), ctypes.byref(d)))
            return d.value
        _check(load().gks_step(self._h, int(n), None))
        return None

    def batch_step(self, n=1):
        _check(load().gks_batch_step(self._h, int(n)))

    def read(self):
        T = self.mesh.n_tri
        W = np.zeros((6, T))
        gW = np.zeros((6, 2, T))
        t = ctypes.c_double()
        _check(load().gks_state_read(self._h, _d(W), _d(gW), ctypes.byref(t)))
        return W, gW, t.value

    def time(self, s=0):
        t, dt = ctypes.c_double(), ctypes.c_double()
        _check(load().gks_state_time(self._h, int(s), ctypes.byref(t), ctypes.byref(dt)))
        return t.value, dt.value

    def mass(self, s=-1):
        m = np.zeros(2)
        _check(load().gks_state_mass(self._h, int(s), _d(m)))
        return m

    DIAGNOSTICS = ("t", "dt", "mass_upper", "mass_lower", "max_speed_upper", "max_speed_lower",
                   "spread_eta1", "spread_eta2")

    def diagnostics(self, s=0):
        """Per-step diagnostics of scenario s from device reductions (see gks_state_diagnostics):
        time, last step, layer masses, largest layer speeds, spreads of the two levels."""
        out = np.zeros(8)
        _check(load().gks_state_diagnostics(self._h, int(s), _d(out)))
        return dict(zip(self.DIAGNOSTICS, out.tolist()))

    def run_logged(self, n_steps, out, every=1, s=0):
        """Advance n_steps steps, writing every `every` steps one JSON line of diagnostics of
        scenario s (plus the share of cells the learned indicator skipped, when it is on) to the
        text stream `out`; returns the last record."""
        rec = None
        done = 0
        while done < n_steps:
            k = min(every, n_steps - done)
            self.step(k)
            done += k
            rec = {"step": done, **self.diagnostics(s)}
            if getattr(self, "_ind_params", None) is not None:
                rec["skipped_fraction"] = self.indicator_eval()[2] / self.mesh.n_tri
            out.write(json.dumps(rec) + "\n")
        return rec

    def check(self):
        """First cell updated to a non-finite or non-positive-thickness state, or -1 (no raise)."""
        first = ctypes.c_int64(-1)
        code = load().gks_state_check(self._h, ctypes.byref(first))
        if code not in (GKS_OK, GKS_ENONFINITE):
            _check(code)
        return first.value

    def save(self):
        """Checkpoint of the state as bytes (see gks_state_save)."""
        n = ctypes.c_int64()
        _check(load().gks_state_checkpoint_size(self._h, ctypes.byref(n)))
        blob = np.zeros(n.value, dtype=np.uint8)
        _check(load().gks_state_save(self._h, blob.ctypes.data_as(_vp), blob.nbytes))
        return blob.tobytes()

    def load(self, blob):
        buf = np.frombuffer(blob, dtype=np.uint8).copy()
        _check(load().gks_state_load(self._h, buf.ctypes.data_as(_vp), buf.nbytes))

    def buffer(self, name):
        """Intermediate array of the last stage (see gks_buffer in include/gks.h)."""
        which, rows, fp64 = BUFFERS[name]
        n = self.mesh.n_edges if name in ("eoh", "eom") else self.mesh.n_tri
        if fp64 is None:
            dt = np.uint8
        else:
            dt = np.float64 if (fp64 or self._params[0].precision == GKS_FP64) else np.float32
        out = np.zeros((rows, n), dtype=dt)
        _check(load().gks_state_buffer(self._h, which, out.ctypes.data_as(_vp), out.nbytes))
        return out

    def autotune(self, reps=3):
        """Pick the threads per block of the edge and cell kernels by timing; returns
        {kernel class: threads per block}.  The state's values are restored."""
        out = (ctypes.c_int32 * len(KERNELS))()
        _check(load().gks_autotune(self._h, int(reps), out))
        return dict(zip(KERNELS, list(out)))

    def profile(self, enable=True):
        _check(load().gks_profile(self._h, int(bool(enable))))

    def profile_read(self):
        """{kernel: (total_ms, launches)} for every kernel class."""
        out = {}
        for k, name in enumerate(KERNELS):
            ms, n = ctypes.c_double(), ctypes.c_int64()
            _check(load().gks_profile_read(self._h, k, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    # learned smoothness indicator
    def indicator(self, params, threshold=0.0):
        """Switch the indicator on (params [7105]) or off (params None) for later stages."""
        if params is None:
            _check(load().gks_indicator_set(self._h, None, 0.0))
            self._ind_params = None
            return
        self._ind_params = _f32(params)
        if self._ind_params.size != MLP_PARAMS:
            raise ValueError(f"{MLP_PARAMS} parameters expected")
        _check(load().gks_indicator_set(self._h, _pf(self._ind_params), float(threshold)))

    def indicator_eval(self):
        """(logits [T], mask [T], n_skip) of the latest state."""
        T = self.mesh.n_tri
        z = np.zeros(T, dtype=np.float32)
        m = np.zeros(T, dtype=np.uint8)
        k = ctypes.c_int64()
        _check(load().gks_indicator_eval(self._h, _pf(z), _pu8(m), ctypes.byref(k)))
        return z, m, k.value

    def features(self):
        X = np.zeros((self.mesh.n_tri, MLP_FEATURES), dtype=np.float32)
        _check(load().gks_state_features(self._h, _pf(X)))
        return X

    def labels(self, tol=1e-7):
        y = np.zeros(self.mesh.n_tri, dtype=np.uint8)
        _check(load().gks_state_labels(self._h, float(tol), _pu8(y)))
        return y

    def close(self):
        if getattr(self, "_h", None):
            load().gks_state_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit the module's globals may already be gone; the process's end frees
        # the device memory then
        if not _finalizing():
            self.close()


class Trainer:
    """Device-resident sample set and parameters of the indicator network (see include/gks.h)."""

    def __init__(self, capacity, params0, max_batch=4096, stream=None):
        lib = load()
        p0 = _f32(params0)
        if p0.size != MLP_PARAMS:
            raise ValueError(f"{MLP_PARAMS} parameters expected")
        if stream is None:
            stream = current_stream()
        h = _vp()
        _check(lib.gks_trainer_create(int(capacity), int(max_batch), _pf(p0), stream, ctypes.byref(h)))
        self._h = h

    def add(self, X, y):
        X = _f32(X).reshape(-1, MLP_FEATURES)
        y = np.ascontiguousarray(y, dtype=np.uint8)
        _check(load().gks_trainer_add(self._h, _pf(X), _pu8(y), X.shape[0]))

    def add_state(self, state, tol=1e-7):
        n = ctypes.c_int64()
        _check(load().gks_trainer_add_state(self._h, state._h, float(tol), ctypes.byref(n)))
        return n.value

    def info(self):
        n, p = ctypes.c_int64(), ctypes.c_int64()
        _check(load().gks_trainer_info(self._h, ctypes.byref(n), ctypes.byref(p)))
        return n.value, p.value

    def grad(self, idx):
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        loss = ctypes.c_float()
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        _check(load().gks_trainer_grad(self._h, idx.ctypes.data_as(_i32p), idx.size, ctypes.byref(loss), _pf(g)))
        return loss.value, g

    def fit(self, epochs, batch=1024, lr=1e-3, seed=0):
        out = np.zeros(max(int(epochs), 1), dtype=np.float32)
        _check(load().gks_trainer_fit(self._h, int(epochs), int(batch), float(lr), ctypes.c_uint64(seed), _pf(out)))
        return out[:int(epochs)]

    def params(self):
        P = np.zeros(MLP_PARAMS, dtype=np.float32)
        _check(load().gks_trainer_params(self._h, _pf(P)))
        return P

    def logits(self):
        n, _ = self.info()
        z = np.zeros(n, dtype=np.float32)
        _check(load().gks_trainer_logits(self._h, _pf(z)))
        return z

    def threshold(self, max_false_skip=1e-4):
        t = ctypes.c_float()
        _check(load().gks_trainer_threshold(self._h, float(max_false_skip), ctypes.byref(t)))
        return t.value

    def close(self):
        if getattr(self, "_h", None):
            load().gks_trainer_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit the module's globals may already be gone; the process's end frees
        # the device memory then
        if not _finalizing():
            self.close()
