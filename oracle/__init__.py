"""FP64 CPU oracle of the sparse D3Q19 LBGK update -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU legs (the CPU
baseline and the oracle timing table) may import this package.  It shares no code with the GPU library; the only thing
both consume is the geometry produced by the seeded input generators.

Thin ctypes marshalling over ``oracle.c`` (plain C, FP64, array-of-structures,
push order, input site order).  Geometry objects are duck-typed: anything with
``coords`` (n,3) int32, ``nbr`` (n,19) int32 and ``iolets`` (objects with
kind, role, centre, normal, radius, vdir, table).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# The mutation tests build altered copies of the sources elsewhere and point
# the package at them through these two variables.
_SRC = os.environ.get("HLB_ORACLE_SRC", _HERE)
_SO = os.environ.get("HLB_ORACLE_LIB", os.path.join(_HERE, "liboracle.so"))
_lib = None
Q = 19


def build(verbose: bool = False) -> str:
    """Compile liboracle.so (gcc, -O2, no FP contraction, OpenMP)."""
    srcs = [os.path.join(_SRC, s) for s in ("oracle.c", "oracle_adjoint.c", "oracle_tangent.c")]
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           *srcs, "-o", _SO, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return _SO


class _Iolet(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("role", ctypes.c_int32), ("centre", ctypes.c_double * 3),
                ("normal", ctypes.c_double * 3), ("radius", ctypes.c_double), ("vdir", ctypes.c_double * 3),
                ("table", ctypes.c_void_p), ("table_len", ctypes.c_int64), ("rho_local", ctypes.c_int32)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    P, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.orc_lattice.argtypes = [P, P, P]
    lib.orc_equilibrium.argtypes = [d, P, P]
    lib.orc_moments.argtypes = [P, P, P]
    lib.orc_collide.argtypes = [P, d, P]
    lib.orc_init.argtypes = [i64, P, P, d, P]
    lib.orc_step.argtypes = [i64, P, P, d, d, P, i32, P, i64, P, P, P, P]
    lib.orc_step.restype = ctypes.c_int
    lib.orc_run.argtypes = [i64, P, P, d, d, P, i32, P, i64, i64, P, P, P]
    lib.orc_run.restype = ctypes.c_int
    lib.orc_macros.argtypes = [i64, P, d, P, P, P, P]
    lib.orc_mass.argtypes = [i64, P]
    lib.orc_mass.restype = d
    lib.orc_wss_sum.argtypes = [i64, P, d, P]
    lib.orc_wss_sum.restype = d
    lib.orc_threads.argtypes = []
    lib.orc_threads.restype = ctypes.c_int32
    lib.orc_set_threads.argtypes = [ctypes.c_int32]
    lib.orc_set_threads.restype = None
    if hasattr(lib, "orc_adj_run"):
        _declare_adjoint(lib)
    _lib = lib
    return lib


def _declare_adjoint(lib):
    P, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.orc_adj_run.argtypes = [i64, P, P, d, d, P, i32, P, i64, i64, i64, i64, i32, P, P, P, P, P, P]
    lib.orc_adj_run.restype = ctypes.c_int
    lib.orc_adj_run_wk.argtypes = [i64, P, P, d, d, P, i32, P, i64, i64, i64, i64, i32, P, P, P, P, P, P, P, P]
    lib.orc_adj_run_wk.restype = ctypes.c_int
    lib.orc_tl_run.argtypes = [i64, P, P, d, d, P, i32, P, i64, i64, i64, i64, i32, P, P, P, P, P, P]
    lib.orc_tl_run.restype = ctypes.c_int
    lib.orc_iolet_flux.argtypes = [i64, P, P, d, d, P, i32, i64, P, P]
    lib.orc_iolet_flux.restype = ctypes.c_int


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c64(a, dtype=np.float64):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


class Problem:
    """A geometry plus the physics parameters the oracle needs, marshalled once."""

    def __init__(self, geom, tau: float, rho0: float = 1.0, tables=None, phi=None, ladd_rho_local: bool = False):
        """ladd_rho_local: the Ladd rule takes each site's own density at t
        instead of rho0 (forward update only)."""
        self.ladd_rho_local = bool(ladd_rho_local)
        self.n = int(geom.coords.shape[0])
        self.coords = np.ascontiguousarray(geom.coords, dtype=np.int32)
        self.nbr = np.ascontiguousarray(geom.nbr, dtype=np.int32)
        self.tau = float(tau)
        self.rho0 = float(rho0)
        self.phi = _c64(phi)
        self._tables = []
        ios = (_Iolet * max(1, len(geom.iolets)))()
        for k, io in enumerate(geom.iolets):
            tab = tables[k] if tables is not None and tables[k] is not None else io.table
            if tab is None:
                tab = np.array([0.0 if io.kind == 0 else self.rho0])
            tab = np.ascontiguousarray(tab, dtype=np.float64).reshape(-1)
            self._tables.append(tab)
            ios[k].kind = int(io.kind)
            ios[k].role = int(io.role)
            ios[k].centre[:] = [float(v) for v in io.centre]
            ios[k].normal[:] = [float(v) for v in io.normal]
            ios[k].radius = float(io.radius)
            vd = getattr(io, "vdir", (0.0, 0.0, 0.0)) or (0.0, 0.0, 0.0)
            ios[k].vdir[:] = [float(v) for v in vd]
            ios[k].table = tab.ctypes.data_as(ctypes.c_void_p)
            ios[k].table_len = tab.size
            ios[k].rho_local = 1 if (self.ladd_rho_local and int(io.kind) == 0) else 0
        self.io = ios
        self.n_io = len(geom.iolets)

    # -- state ---------------------------------------------------------
    def init(self, rho=None, u=None) -> np.ndarray:
        f = np.empty((self.n, Q), dtype=np.float64)
        _load().orc_init(self.n, _p(_c64(rho)), _p(_c64(u)), self.rho0, _p(f))
        return f

    def step(self, f, t: int, write_count: bool = False):
        f = np.ascontiguousarray(f, dtype=np.float64)
        F = np.full_like(f, np.nan)
        flux = np.zeros(1)
        wc = np.zeros((self.n, Q), dtype=np.int32) if write_count else None
        rc = _load().orc_step(self.n, _p(self.coords), _p(self.nbr), self.tau, self.rho0, ctypes.byref(self.io),
                              self.n_io, _p(self.phi), int(t), _p(f), _p(F), _p(flux), _p(wc))
        if rc != 0:
            raise ValueError("oracle step: bad link code")
        return (F, float(flux[0]), wc) if write_count else (F, float(flux[0]))

    def run(self, f, t0: int, nsteps: int):
        """Advance f (in place) from t0 by nsteps; returns the summed boundary flux."""
        assert f.dtype == np.float64 and f.flags.c_contiguous and f.shape == (self.n, Q)
        work = np.empty_like(f)
        flux = np.zeros(1)
        rc = _load().orc_run(self.n, _p(self.coords), _p(self.nbr), self.tau, self.rho0, ctypes.byref(self.io),
                             self.n_io, _p(self.phi), int(t0), int(nsteps), _p(f), _p(work), _p(flux))
        if rc != 0:
            raise ValueError("oracle run: bad link code")
        return float(flux[0])

    def macros(self, f):
        rho = np.empty(self.n)
        u = np.empty((self.n, 3))
        wss = np.empty(self.n)
        _load().orc_macros(self.n, _p(self.nbr), self.tau, _p(np.ascontiguousarray(f)), _p(rho), _p(u), _p(wss))
        return rho, u, wss

    def mass(self, f) -> float:
        return float(_load().orc_mass(self.n, _p(np.ascontiguousarray(f))))

    def wss_sum(self, f) -> float:
        return float(_load().orc_wss_sum(self.n, _p(self.nbr), self.tau, _p(np.ascontiguousarray(f))))

    def adjoint(self, f0, t0: int, nsteps: int, obj_t0: int, obj_t1: int, weights=None, state_grad=False,
                windkessel=None):
        """Reference adjoint (oracle_adjoint.c).  J = sum over t in (obj_t0,
        obj_t1] of the summed wall shear stress (weights None), or of
        sum_k weights[k] Q_k(t), Q_k(t) the outflow of iolet k during the
        update t-1 -> t (weights [n_io]).  Returns J, the derivatives with
        respect to the per-step iolet table values [n_io][nsteps] (amplitude
        or ghost density) and the per-site porosity [n], and with
        state_grad also the derivative with respect to f0 [n][19].  Keeps all
        nsteps+1 states in memory.  windkessel maps pressure iolets to
        (rho_ref, R1, C, R2, X0) as in run_windkessel; their densities then
        come from that model, and their table-value derivatives are those
        with respect to the density held at each step."""
        if self.ladd_rho_local:
            raise ValueError("the reference adjoint takes the Ladd rule with rho0")
        f0 = np.ascontiguousarray(f0, dtype=np.float64)
        J = np.zeros(1)
        dA = np.zeros((max(self.n_io, 1), nsteps))
        dphi = np.zeros(self.n)
        w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
        df0 = np.zeros_like(f0) if state_grad else None
        if windkessel:
            on = np.zeros(max(self.n_io, 1), dtype=np.int32)
            par = np.zeros((max(self.n_io, 1), 5))
            for k, m in windkessel.items():
                on[k] = 1
                par[k] = m
            rc = _load().orc_adj_run_wk(self.n, _p(self.coords), _p(self.nbr), self.tau, self.rho0,
                                        ctypes.byref(self.io), self.n_io, _p(self.phi), int(t0), int(nsteps),
                                        int(obj_t0), int(obj_t1), 0 if w is None else 1,
                                        None if w is None else _p(w), _p(on), _p(par), _p(f0),
                                        _p(J), _p(dA), _p(dphi), _p(df0))
        else:
            rc = _load().orc_adj_run(self.n, _p(self.coords), _p(self.nbr), self.tau, self.rho0,
                                     ctypes.byref(self.io), self.n_io, _p(self.phi), int(t0), int(nsteps),
                                     int(obj_t0), int(obj_t1), 0 if w is None else 1, None if w is None else _p(w),
                                     _p(f0), _p(J), _p(dA), _p(dphi), _p(df0))
        if rc != 0:
            raise ValueError("oracle adjoint failed")
        if state_grad:
            return float(J[0]), dA[: self.n_io], dphi, df0
        return float(J[0]), dA[: self.n_io], dphi

    def tangent(self, f0, t0: int, nsteps: int, obj_t0: int, obj_t1: int, weights=None, df0=None, dtab=None,
                dphi=None) -> float:
        """Tangent-linear model (oracle_tangent.c): the derivative of the
        objective of adjoint() in the direction (df0 [n][19], dtab
        [n_io][nsteps], dphi [n]); each part may be None (zero)."""
        if self.ladd_rho_local:
            raise ValueError("the tangent-linear model takes the Ladd rule with rho0")
        f0 = np.ascontiguousarray(f0, dtype=np.float64)
        dJ = np.zeros(1)
        w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
        if dtab is not None:
            dtab = np.ascontiguousarray(dtab, dtype=np.float64)
            assert dtab.shape == (self.n_io, nsteps)
        rc = _load().orc_tl_run(self.n, _p(self.coords), _p(self.nbr), self.tau, self.rho0, ctypes.byref(self.io),
                                self.n_io, _p(self.phi), int(t0), int(nsteps), int(obj_t0), int(obj_t1),
                                0 if w is None else 1, None if w is None else _p(w), _p(f0), _p(_c64(df0)),
                                _p(dtab), _p(_c64(dphi)), _p(dJ))
        if rc != 0:
            raise ValueError("oracle tangent failed")
        return float(dJ[0])

    def iolet_flux(self, f, t: int) -> np.ndarray:
        """Outflow of each iolet during the update t -> t+1 from the state f at t."""
        Q = np.zeros(max(self.n_io, 1))
        f = np.ascontiguousarray(f, dtype=np.float64)
        rc = _load().orc_iolet_flux(self.n, _p(self.coords), _p(self.nbr), self.tau, self.rho0,
                                    ctypes.byref(self.io), self.n_io, int(t), _p(f), _p(Q))
        if rc != 0:
            raise ValueError("bad link code")
        return Q[: self.n_io]

    def set_table(self, k: int, values):
        """Replace iolet k's per-step table."""
        tab = np.ascontiguousarray(values, dtype=np.float64).reshape(-1)
        self._tables[k] = tab
        self.io[k].table = tab.ctypes.data_as(ctypes.c_void_p)
        self.io[k].table_len = tab.size

    def run_windkessel(self, f, t0: int, nsteps: int, models: dict) -> dict:
        """nsteps updates from time t0 with Windkessel outlets.  models maps a
        pressure iolet k to (rho_ref, R1, C, R2, X0): the update s -> s+1
        uses rho_k(s); its outflow Q_k(s) (iolet_flux) then gives
          X(s+1) = X(s) + (Q - X/R2)/C  (C > 0; no X/R2 term if R2 = 0),
                   R2 Q                  (C = 0),
          rho_k(s+1) = rho_ref + R1 Q + X(s+1).
        f is advanced in place; returns {k: (rho_next, X, Q_last)}."""
        st = {k: [m[4], m[0] + m[4], 0.0] for k, m in models.items()}
        for s in range(nsteps):
            t = t0 + s
            for k in models:
                self.set_table(k, [st[k][1]])
            Q = self.iolet_flux(f, t)
            self.run(f, t, 1)
            for k, (rho_ref, R1, C, R2, _) in models.items():
                X = st[k][0]
                X = X + (Q[k] - (X / R2 if R2 > 0 else 0.0)) / C if C > 0 else R2 * Q[k]
                st[k] = [X, rho_ref + R1 * Q[k] + X, Q[k]]
        return {k: (v[1], v[0], v[2]) for k, v in st.items()}

    def objective(self, f0, t0: int, nsteps: int, obj_t0: int, obj_t1: int, weights=None,
                  windkessel=None) -> float:
        """J of adjoint() by a plain forward run (no derivatives); windkessel
        as in adjoint() (the outlets' tables are put back afterwards)."""
        f = np.array(f0, dtype=np.float64, copy=True)
        wk = dict(windkessel or {})
        saved = {k: self._tables[k].copy() for k in wk}
        st = {k: [m[4], m[0] + m[4]] for k, m in wk.items()}  # X, rho
        J = 0.0
        for s in range(nsteps):
            t = t0 + s + 1
            for k in wk:
                self.set_table(k, [st[k][1]])
            flux_here = weights is not None and obj_t0 < t <= obj_t1
            Q = self.iolet_flux(f, t - 1) if (flux_here or wk) else None
            if flux_here:
                J += float(np.dot(weights, Q))
            self.run(f, t0 + s, 1)
            if weights is None and obj_t0 < t <= obj_t1:
                J += self.wss_sum(f)
            for k, (rho_ref, R1, C, R2, _) in wk.items():
                X = st[k][0]
                X = X + (Q[k] - (X / R2 if R2 > 0 else 0.0)) / C if C > 0 else R2 * Q[k]
                st[k] = [X, rho_ref + R1 * Q[k] + X]
        for k, tab in saved.items():
            self.set_table(k, tab)
        return J

    def collide_all(self, f) -> np.ndarray:
        out = np.empty_like(f)
        for x in range(self.n):
            out[x] = collide(f[x], self.tau)
        return out


def threads() -> int:
    return int(_load().orc_threads())


def set_threads(n: int):
    """Use n OpenMP threads in the oracle from now on."""
    _load().orc_set_threads(int(n))


# -- single-site functions -------------------------------------------------

def lattice():
    c = np.empty((Q, 3), dtype=np.int32)
    w = np.empty(Q)
    opp = np.empty(Q, dtype=np.int32)
    _load().orc_lattice(_p(c), _p(w), _p(opp))
    return c, w, opp


def equilibrium(rho: float, u) -> np.ndarray:
    out = np.empty(Q)
    _load().orc_equilibrium(float(rho), _p(_c64(u)), _p(out))
    return out


def moments(f):
    rho = np.zeros(1)
    u = np.empty(3)
    _load().orc_moments(_p(_c64(f)), _p(rho), _p(u))
    return float(rho[0]), u


def collide(f, tau: float) -> np.ndarray:
    out = np.empty(Q)
    _load().orc_collide(_p(_c64(f)), float(tau), _p(out))
    return out
