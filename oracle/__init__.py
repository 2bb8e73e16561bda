"""FP64 CPU oracle of the mEVP momentum subcycle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. It wraps ``liboracle_mevp.so`` (plain C, built by
``oracle/build.py``) with numpy arrays. See ``mevp_oracle.h`` for the layouts
and ``mevp_oracle.c`` for the readings of the paper it follows.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, asdict

import numpy as np

from . import build as _build

_lib = None


#: a different build of the oracle's source to load instead of the default one;
#: set only by the mutation test, which plants mistakes in copies of the source
#: and checks that the pins reject each of them
ENV_LIB = "MEVP_ORACLE_LIB"


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get(ENV_LIB) or _build.LIB
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        L.or_mesh_create.restype = C.c_void_p
        L.or_mesh_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, dp]
        L.or_mesh_create_iso.restype = C.c_void_p
        L.or_mesh_create_iso.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, dp]
        L.or_mesh_destroy.argtypes = [C.c_void_p]
        L.or_tables.restype = C.c_int
        L.or_tables.argtypes = [C.c_int, C.c_int] + [dp] * 7
        L.or_element_geometry.argtypes = [C.c_void_p, C.c_int, dp, dp, dp]
        L.or_node_masses.argtypes = [C.c_void_p, C.c_void_p, dp, dp, dp, dp]
        L.or_air_stress.argtypes = [C.c_void_p, C.c_int, dp, dp]
        L.or_strain.argtypes = [C.c_void_p, dp, dp]
        L.or_stress.argtypes = [C.c_void_p, C.c_void_p, dp, dp, dp, dp]
        L.or_divergence.argtypes = [C.c_void_p, dp, dp]
        L.or_velocity.argtypes = [C.c_void_p, C.c_void_p] + [dp] * 7
        L.or_step.restype = C.c_int
        L.or_step.argtypes = [C.c_void_p, C.c_void_p, dp, dp, dp, dp, dp, dp, C.c_int]
        L.or_subcycles.restype = C.c_int
        L.or_subcycles.argtypes = [C.c_void_p, C.c_void_p] + [dp] * 7 + [C.c_int]
        L.or_strain_gauss.argtypes = [C.c_void_p, dp, dp]
        L.or_eval_gauss.argtypes = [C.c_void_p, dp, C.c_int, dp]
        L.or_stress_gauss.argtypes = [C.c_void_p, C.c_void_p, dp, dp, dp, dp, dp, dp]
        L.or_project.argtypes = [C.c_void_p, dp, C.c_int, dp]
        L.or_num_threads.restype = C.c_int
        L.or_set_num_threads.argtypes = [C.c_int]
        L.or_advect.argtypes = [C.c_void_p, C.c_double, dp, dp, dp]
        L.or_advect_rate.argtypes = [C.c_void_p, dp, dp, dp]
        _lib = L
    return _lib


class _Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("Pstar", "C", "DeltaMin", "alpha", "beta", "rho_i",
                                          "rho_a", "C_a", "rho_o", "C_o", "f_cor", "dt")] + \
               [("relax_form", C.c_int)]


@dataclass
class Params:
    """Physical and iteration parameters. P*, C, alpha, beta, n_sub and dt follow
    the paper (Listing 1, Sec. 2, Sec. 4); the remaining values are conventional
    viscous-plastic constants (the paper states none)."""
    Pstar: float = 27500.0
    C: float = 20.0
    DeltaMin: float = 2e-9
    alpha: float = 300.0
    beta: float = 300.0
    rho_i: float = 900.0
    rho_a: float = 1.3
    C_a: float = 1.2e-3
    rho_o: float = 1026.0
    C_o: float = 5.5e-3
    f_cor: float = 1.46e-4
    dt: float = 120.0
    relax_form: int = 0

    def _c(self):
        return _Params(**asdict(self))


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Mesh:
    """Oracle mesh: nx x ny quads, DG stress with ns dofs, DG ice fields with na dofs.
    Geometry from the cell vertices [2][(nx+1)(ny+1)] (bilinear map) or, with
    ``nodes`` [2][(2nx+1)(2ny+1)], from the CG2 node positions (isoparametric map)."""

    def __init__(self, nx, ny, ns, na, vertices=None, nodes=None):
        self.nx, self.ny, self.ns, self.na = nx, ny, ns, na
        if (vertices is None) == (nodes is None):
            raise ValueError("give exactly one of vertices and nodes")
        if nodes is not None:
            self.nodes = _f64(nodes)
            if self.nodes.shape != (2, (2 * nx + 1) * (2 * ny + 1)):
                raise ValueError("nodes must be [2][(2nx+1)(2ny+1)]")
            self._h = lib().or_mesh_create_iso(nx, ny, ns, na, _p(self.nodes))
        else:
            self.vertices = _f64(vertices)
            if self.vertices.shape != (2, (nx + 1) * (ny + 1)):
                raise ValueError("vertices must be [2][(nx+1)(ny+1)]")
            self._h = lib().or_mesh_create(nx, ny, ns, na, _p(self.vertices))
        if not self._h:
            raise ValueError("oracle rejected the mesh (sizes, ns/na or a non-positive Jacobian)")
        self.ng = 4 if ns == 3 else 9

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.or_mesh_destroy(h)
            self._h = None

    @property
    def ne(self):
        return self.nx * self.ny

    @property
    def nn(self):
        return (2 * self.nx + 1) * (2 * self.ny + 1)

    # --- per time step -------------------------------------------------
    def node_masses(self, p: Params, H, A):
        MH = np.zeros(self.nn)
        mA = np.zeros(self.nn)
        H, A = _f64(H), _f64(A)
        pc = p._c()
        lib().or_node_masses(self._h, C.byref(pc), _p(H), _p(A), _p(MH), _p(mA))
        return MH, mA

    def air_stress(self, p: Params, wind):
        wind = _f64(wind)
        tau = np.zeros((2, self.nn))
        pc = p._c()
        lib().or_air_stress(C.byref(pc), self.nn, _p(wind), _p(tau))
        return tau

    # --- phases --------------------------------------------------------
    def strain(self, v):
        v = _f64(v)
        E = np.zeros((3, self.ns, self.ne))
        lib().or_strain(self._h, _p(v), _p(E))
        return E

    def stress(self, p: Params, E, H, A, S):
        E, H, A = _f64(E), _f64(H), _f64(A)
        S = _f64(S).copy()
        pc = p._c()
        lib().or_stress(self._h, C.byref(pc), _p(E), _p(H), _p(A), _p(S))
        return S

    def divergence(self, S):
        S = _f64(S)
        F = np.zeros((2, self.nn))
        lib().or_divergence(self._h, _p(S), _p(F))
        return F

    def velocity(self, p: Params, F, MH, mA, tau, ocean, vn, v):
        v = _f64(v).copy()
        F, MH, mA, tau, ocean, vn = map(_f64, (F, MH, mA, tau, ocean, vn))
        pc = p._c()
        lib().or_velocity(self._h, C.byref(pc), _p(F), _p(MH), _p(mA), _p(tau), _p(ocean),
                          _p(vn), _p(v))
        return v

    # --- drivers -------------------------------------------------------
    def step(self, p: Params, H, A, wind, ocean, v, S, n_sub):
        """One time step (snapshot v^n, then n_sub subcycles); returns new (v, S)."""
        v = _f64(v).copy()
        S = _f64(S).copy()
        H, A, wind, ocean = map(_f64, (H, A, wind, ocean))
        pc = p._c()
        rc = lib().or_step(self._h, C.byref(pc), _p(H), _p(A), _p(wind), _p(ocean), _p(v), _p(S),
                           int(n_sub))
        if rc != 0:
            raise RuntimeError(f"or_step failed ({rc})")
        return v, S

    def subcycles(self, p: Params, H, A, wind, ocean, vn, v, S, n_sub):
        v = _f64(v).copy()
        S = _f64(S).copy()
        H, A, wind, ocean, vn = map(_f64, (H, A, wind, ocean, vn))
        pc = p._c()
        rc = lib().or_subcycles(self._h, C.byref(pc), _p(H), _p(A), _p(wind), _p(ocean), _p(vn),
                                _p(v), _p(S), int(n_sub))
        if rc != 0:
            raise RuntimeError(f"or_subcycles failed ({rc})")
        return v, S

    def run(self, p: Params, H, A, wind, ocean, n_steps, n_sub, v=None, S=None):
        v = np.zeros((2, self.nn)) if v is None else _f64(v).copy()
        S = np.zeros((3, self.ns, self.ne)) if S is None else _f64(S).copy()
        for _ in range(n_steps):
            v, S = self.step(p, H, A, wind, ocean, v, S, n_sub)
        return v, S

    def advect(self, dt, v, H, A):
        """One advection step of H and A (returns new arrays)."""
        v = _f64(v)
        H = _f64(H).copy()
        A = _f64(A).copy()
        lib().or_advect(self._h, float(dt), _p(v), _p(H), _p(A))
        return H, A

    # --- test hooks ----------------------------------------------------
    def advect_rate(self, v, U):
        v, U = _f64(v), _f64(U)
        L = np.zeros((self.na, self.ne))
        lib().or_advect_rate(self._h, _p(v), _p(U), _p(L))
        return L

    def element_geometry(self, e):
        wd = np.zeros(self.ng)
        gx = np.zeros((9, self.ng))
        gy = np.zeros((9, self.ng))
        lib().or_element_geometry(self._h, int(e), _p(wd), _p(gx), _p(gy))
        return wd, gx, gy

    def strain_gauss(self, v):
        v = _f64(v)
        eps = np.zeros((3, self.ng, self.ne))
        lib().or_strain_gauss(self._h, _p(v), _p(eps))
        return eps

    def eval_gauss(self, coef):
        coef = _f64(coef)
        nc = coef.shape[0]
        out = np.zeros((nc, self.ng, self.ne))
        lib().or_eval_gauss(self._h, _p(coef), nc, _p(out))
        return out

    def stress_gauss(self, p: Params, E, H, A):
        E, H, A = _f64(E), _f64(H), _f64(A)
        s = np.zeros((3, self.ng, self.ne))
        P = np.zeros((self.ng, self.ne))
        D = np.zeros((self.ng, self.ne))
        pc = p._c()
        lib().or_stress_gauss(self._h, C.byref(pc), _p(E), _p(H), _p(A), _p(s), _p(P), _p(D))
        return s, P, D

    def project(self, g):
        g = _f64(g)
        nc = g.shape[0]
        out = np.zeros((nc, self.ns, self.ne))
        lib().or_project(self._h, _p(g), nc, _p(out))
        return out


def tables(ns, na=1):
    """Reference tables: (gpts, gwts, psiS[ns][nG], psiA[na][nG], phi, dxi, deta [9][nG])."""
    ngp = 2 if ns == 3 else 3
    ng = ngp * ngp
    gp, gw = np.zeros(ngp), np.zeros(ngp)
    psiS, psiA = np.zeros((ns, ng)), np.zeros((na, ng))
    phi, dxi, deta = np.zeros((9, ng)), np.zeros((9, ng)), np.zeros((9, ng))
    rc = lib().or_tables(ns, na, _p(gp), _p(gw), _p(psiS), _p(psiA), _p(phi), _p(dxi), _p(deta))
    if rc < 0:
        raise ValueError("bad ns")
    return gp, gw, psiS, psiA, phi, dxi, deta


def num_threads():
    return lib().or_num_threads()


def set_num_threads(n: int):
    """Threads of the following oracle calls (results do not depend on it)."""
    lib().or_set_num_threads(int(n))
