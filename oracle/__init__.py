"""Python access to the FP64 CPU oracle (test infrastructure only).

The oracle is a plain C implementation of the compact gas-kinetic scheme for the two-layer shallow
water equations, written from the paper independently of the HIP library.  Only the tests, the
smoke check and the CPU-baseline leg of the benchmark use it.  ``build()`` compiles it with gcc;
``load()`` returns the ctypes handle, building on first use if the shared object is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gks_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


class Params(ctypes.Structure):
    _fields_ = [("G", ctypes.c_double), ("chi", ctypes.c_double), ("cfl", ctypes.c_double),
                ("eps", ctypes.c_double), ("eps_num", ctypes.c_double), ("linear", ctypes.c_int),
                ("per_side_gb", ctypes.c_int), ("alpha_mode", ctypes.c_int), ("src_order", ctypes.c_int),
                ("grad_mode", ctypes.c_int), ("h_dry", ctypes.c_double)]


def build() -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.om_mesh_new.restype = ctypes.c_void_p
    lib.om_mesh_new.argtypes = [_dp, ctypes.c_int, _ip, ctypes.c_int, _dp, ctypes.c_int,
                                ctypes.c_double, ctypes.c_double]
    lib.om_mesh_free.argtypes = [ctypes.c_void_p]
    lib.om_mesh_n_edges.argtypes = [ctypes.c_void_p]
    lib.om_mesh_n_edges.restype = ctypes.c_int
    lib.om_stencil.argtypes = [ctypes.c_void_p, ctypes.c_int, _ip, _dp]
    lib.om_lsq_matrix.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
    lib.om_reconstruct_cell.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_double,
                                        _dp, _dp, _dp]
    lib.om_gks_point.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, _dp, _dp, _dp, _dp]
    lib.om_gks_point_mode.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int, _dp, _dp, _dp, _dp]
    lib.om_gks_point_integrated.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
    lib.om_moments.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, _dp]
    lib.om_time_integrals.argtypes = [ctypes.c_double, ctypes.c_double, _dp]
    lib.om_side_rate.argtypes = [_dp, ctypes.c_double, _dp]
    lib.om_cell_velocity.restype = ctypes.c_double
    lib.om_cell_velocity.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.om_gks_point_wd.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp, _dp]
    lib.om_dt.restype = ctypes.c_double
    lib.om_dt.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), _dp]
    lib.om_operator.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_double, _dp, _dp,
                                _dp, _dp, _dp, _dp]
    lib.om_operator_src.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_double, _dp, _dp,
                                    _dp, _dp, _dp, _dp, _dp, _dp]
    lib.om_coupling_correction.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, ctypes.c_int,
                                           ctypes.c_double, _dp]
    lib.om_step.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_double, ctypes.c_int,
                            _dp, _dp, _dp, _dp]
    lib.om_mass.argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.om_s2o4_stage.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp]
    lib.om_s2o4_final.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp, _dp]
    lib.om_cell_geometry.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
    lib.om_edge_height.restype = ctypes.c_double
    lib.om_edge_height.argtypes = [ctypes.c_double] * 7
    lib.om_plane_gradient.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp]
    lib.om_features.argtypes = [ctypes.c_void_p, ctypes.c_double, _dp, _dp, _dp]
    lib.om_mlp_forward.argtypes = [_dp, _dp, ctypes.c_int, _dp]
    lib.om_mlp_grad.argtypes = [_dp, _dp, _dp, ctypes.c_int, _dp]
    lib.om_mlp_forward_bf16.argtypes = [_dp, _dp, ctypes.c_int, _dp]
    lib.om_mlp_grad.restype = ctypes.c_double
    lib.om_set_threads.argtypes = [ctypes.c_int]
    lib.om_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


MLP_IN, MLP_H = 44, 64
MLP_PARAMS = MLP_IN * MLP_H + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1


def features(mesh, W, gW, G=9.81):
    """Indicator features [T, 44] of every cell (see om_features)."""
    X = np.zeros((mesh.n_tri, MLP_IN))
    load().om_features(mesh._h, float(G), _d(_f64(W)), _d(_f64(gW)), _d(X))
    return X


def mlp_forward(P, X):
    X = _f64(X)
    z = np.zeros(X.shape[0])
    load().om_mlp_forward(_d(_f64(P)), _d(X), X.shape[0], _d(z))
    return z


def mlp_forward_bf16(P, X):
    """Logits with the bf16 operand rounding of the matrix-core inference (see om_mlp_forward_bf16)."""
    X = _f64(X)
    z = np.zeros(X.shape[0])
    load().om_mlp_forward_bf16(_d(_f64(P)), _d(X), X.shape[0], _d(z))
    return z


def mlp_grad(P, X, y):
    """(mean logistic loss, gradient [MLP_PARAMS]) of the MLP on the batch (X, y)."""
    X = _f64(X)
    g = np.zeros(MLP_PARAMS)
    loss = load().om_mlp_grad(_d(_f64(P)), _d(X), _d(_f64(y)), X.shape[0], _d(g))
    return loss, g


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Mesh:
    """Oracle mesh: connectivity, stencils and least-squares matrices built in plain C."""

    BC = {"wall": 0, "periodic": 1, "free": 2}

    def __init__(self, node_xy, tri, node_B=None, periodic_L=None, boundary=None):
        lib = load()
        self.node_xy = _f64(node_xy)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32)
        self.node_B = _f64(node_B if node_B is not None else np.zeros(self.node_xy.shape[0]))
        self.n_tri = int(self.tri.shape[0])
        per = periodic_L is not None
        if boundary is None:
            boundary = "periodic" if per else "wall"
        Lx, Ly = (periodic_L if per else (0.0, 0.0))
        self._h = lib.om_mesh_new(_d(self.node_xy), self.node_xy.shape[0],
                                  self.tri.ctypes.data_as(_ip), self.n_tri, _d(self.node_B),
                                  self.BC[boundary], float(Lx), float(Ly))
        if not self._h:
            raise ValueError("oracle rejected the mesh")
        self.n_edges = lib.om_mesh_n_edges(self._h)

    def __del__(self):
        if getattr(self, "_h", None):
            load().om_mesh_free(self._h)
            self._h = None

    @classmethod
    def from_scenario(cls, sc):
        return cls(sc.node_xy, sc.tri, sc.node_B, sc.periodic_L if sc.boundary == "periodic" else None,
                   boundary=sc.boundary)

    def geometry(self):
        a, x, y = (np.zeros(self.n_tri) for _ in range(3))
        load().om_cell_geometry(self._h, _d(a), _d(x), _d(y))
        return a, x, y

    def stencil(self, c):
        cells = np.zeros(10, dtype=np.int32)
        maps = np.zeros((10, 6))
        load().om_stencil(self._h, c, cells.ctypes.data_as(_ip), _d(maps))
        return cells, maps

    def lsq_matrix(self, c):
        M = np.zeros((9, 17))
        load().om_lsq_matrix(self._h, c, _d(M))
        return M

    def plane_gradient(self, c, hk):
        """Gradient of the plane through the values hk[3] at the centres of cell c's local edges
        (edge k joins vertices k and k + 1 of tri[c])."""
        out = np.zeros(2)
        load().om_plane_gradient(self._h, int(c), _d(_f64(hk)), _d(out))
        return out

    def reconstruct(self, c, W, gW, linear=False, G=9.81):
        W, gW = _f64(W), _f64(gW)
        val = np.zeros((6, 6))
        grad = np.zeros((6, 6, 2))
        r0 = np.zeros(6)
        load().om_reconstruct_cell(self._h, c, _d(W), _d(gW), int(linear), float(G), _d(val), _d(grad), _d(r0))
        return val, grad, r0


ALPHA_MODES = {"reading": 0, "paper": 1}


SRC_ORDERS = (2, 4)
# interface values of the gradient update (Sec. 3.3): the continuous evolution solution (the
# paper's choice) or each cell's own side of the interface
GRAD_MODES = {"continuous": 0, "discontinuous": 1}


def params(G=9.81, chi=0.98, cfl=0.3, eps=0.05, eps_num=5.0, linear=False, per_side_gb=False,
           alpha_mode="reading", src_order=2, grad_mode="continuous", h_dry=0.0) -> Params:
    if src_order not in SRC_ORDERS:
        raise ValueError(f"src_order must be one of {SRC_ORDERS}")
    if not h_dry >= 0:
        raise ValueError("h_dry must be >= 0")
    return Params(G, chi, cfl, eps, eps_num, int(linear), int(per_side_gb), ALPHA_MODES[alpha_mode],
                  int(src_order), GRAD_MODES[grad_mode], float(h_dry))


def params_of(sc, linear=False, alpha_mode="reading", src_order=2, grad_mode="continuous", h_dry=None) -> Params:
    """Parameters of a scenario; h_dry defaults to the scenario's own (0 where it has none)."""
    if h_dry is None:
        h_dry = getattr(sc, "h_dry", 0.0)
    return params(G=sc.G, chi=sc.chi, cfl=sc.cfl, linear=linear, alpha_mode=alpha_mode, src_order=src_order,
                  grad_mode=grad_mode, h_dry=h_dry)


def dt(mesh: Mesh, p: Params, W) -> float:
    return load().om_dt(mesh._h, ctypes.byref(p), _d(_f64(W)))


def operator(mesh: Mesh, p: Params, dt_: float, W, gW):
    T = mesh.n_tri
    L, Lt = np.zeros((6, T)), np.zeros((6, T))
    G, Gt = np.zeros((6, 2, T)), np.zeros((6, 2, T))
    load().om_operator(mesh._h, ctypes.byref(p), float(dt_), _d(_f64(W)), _d(_f64(gW)),
                       _d(L), _d(Lt), _d(G), _d(Gt))
    return L, Lt, G, Gt


def coupling_source(mesh: Mesh, p: Params, dt_: float, W, gW):
    """Layer-coupling part of the operator: (S, St), each [4, T] = lower layer x, y, upper x, y."""
    T = mesh.n_tri
    L, Lt = np.zeros((6, T)), np.zeros((6, T))
    G, Gt = np.zeros((6, 2, T)), np.zeros((6, 2, T))
    S, St = np.zeros((4, T)), np.zeros((4, T))
    load().om_operator_src(mesh._h, ctypes.byref(p), float(dt_), _d(_f64(W)), _d(_f64(gW)),
                           _d(L), _d(Lt), _d(G), _d(Gt), _d(S), _d(St))
    return S, St


def coupling_correction(mesh: Mesh, c: int, W, gW, linear=False, G=9.81):
    """Interior correction [8] of the higher-order layer coupling in cell c (om_coupling_correction)."""
    out = np.zeros(8)
    load().om_coupling_correction(mesh._h, int(c), _d(_f64(W)), _d(_f64(gW)), int(linear), float(G), _d(out))
    return out


def step(mesh: Mesh, p: Params, dt_: float, W, gW, nstages: int = 2):
    T = mesh.n_tri
    Wo, gWo = np.zeros((6, T)), np.zeros((6, 2, T))
    load().om_step(mesh._h, ctypes.byref(p), float(dt_), int(nstages), _d(_f64(W)), _d(_f64(gW)),
                   _d(Wo), _d(gWo))
    return Wo, gWo


def run(mesh: Mesh, p: Params, W, gW, t_end: float, max_steps: int = 10 ** 9):
    """Advance to t_end (last step clipped) with the CFL time step; returns (W, gW, t, steps)."""
    t, n = 0.0, 0
    while t < t_end - 1e-14 * max(1.0, t_end) and n < max_steps:
        d = min(dt(mesh, p, W), t_end - t)
        W, gW = step(mesh, p, d, W, gW)
        t += d
        n += 1
    return W, gW, t, n


def s2o4_stage(dt_: float, W, L, Lt):
    """First S2O4 stage on flat arrays: W + dt/2 L + dt^2/8 Lt."""
    W, L, Lt = (_f64(np.ravel(a)) for a in (W, L, Lt))
    out = np.zeros_like(W)
    load().om_s2o4_stage(W.size, float(dt_), _d(W), _d(L), _d(Lt), _d(out))
    return out


def s2o4_final(dt_: float, W, L, Lt, Lt2):
    """Second S2O4 stage on flat arrays: W + dt L + dt^2/6 Lt + dt^2/3 Lt2."""
    W, L, Lt, Lt2 = (_f64(np.ravel(a)) for a in (W, L, Lt, Lt2))
    out = np.zeros_like(W)
    load().om_s2o4_final(W.size, float(dt_), _d(W), _d(L), _d(Lt), _d(Lt2), _d(out))
    return out


def mass(mesh: Mesh, W):
    out = np.zeros(2)
    load().om_mass(mesh._h, _d(_f64(W)), _d(out))
    return out


def moments(U, lam, half, K):
    out = np.zeros(K)
    load().om_moments(float(U), float(lam), int(half), int(K), _d(out))
    return out


def time_integrals(delta, tau):
    out = np.zeros(5)
    load().om_time_integrals(float(delta), float(tau), _d(out))
    return out


def edge_height(zl, zr, hl, hr, unl, unr, G):
    """Interface height of the force model (Sec. 2.3): xi zl + (1 - xi) zr, xi the kinetic fraction
    of the interface Maxwellian moving from the left side to the right."""
    return load().om_edge_height(*(float(x) for x in (zl, zr, hl, hr, unl, unr, G)))


def gks_point(sideL, sideR, G, dt_, eps=0.05, eps_num=5.0, alpha_mode="reading"):
    sL, sR = _f64(sideL), _f64(sideR)
    F0, Ft, Wb, Wbt = (np.zeros(3) for _ in range(4))
    load().om_gks_point_mode(_d(sL), _d(sR), float(G), float(dt_), float(eps), float(eps_num),
                             ALPHA_MODES[alpha_mode], _d(F0), _d(Ft), _d(Wb), _d(Wbt))
    return F0, Ft, Wb, Wbt


def cell_velocity(h, m, h_dry):
    """Velocity of a layer cell (om_cell_velocity): m / h, desingularised below h_dry."""
    return load().om_cell_velocity(float(h), float(m), float(h_dry))


def gks_point_wd(sideL, sideR, G, dt_, h_dry, order1=False, eps=0.05, eps_num=5.0, alpha_mode="reading"):
    sL, sR = _f64(sideL), _f64(sideR)
    F0, Ft, Wb, Wbt = (np.zeros(3) for _ in range(4))
    load().om_gks_point_wd(_d(sL), _d(sR), float(G), float(dt_), float(eps), float(eps_num),
                           ALPHA_MODES[alpha_mode], float(h_dry), int(order1), _d(F0), _d(Ft), _d(Wb), _d(Wbt))
    return F0, Ft, Wb, Wbt


def side_rate(side, G):
    """(h, hU_n, hU_t)_t of one side's own state from its Maxwellian (om_side_rate)."""
    out = np.zeros(3)
    load().om_side_rate(_d(_f64(side)), float(G), _d(out))
    return out


def gks_point_integrated(sideL, sideR, G, delta, tau):
    F = np.zeros(3)
    load().om_gks_point_integrated(_d(_f64(sideL)), _d(_f64(sideR)), float(G), float(delta),
                                   float(tau), _d(F))
    return F
