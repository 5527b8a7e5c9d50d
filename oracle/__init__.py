"""Plain single-threaded FP64 CPU oracle for the GRMHD block update.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``; never by the product package.  The C source
(``orc.c``) shares no code with the HIP path.  Functions here only marshal numpy
arrays into the C library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liborc.so")
_lib = None

MINK, KS = 0, 1
PLM, PPM, PLM_MINMOD, PPM_FLAT = 0, 1, 2, 3
LLF, HLLE = 0, 1
EMF_AVERAGE, EMF_UPWIND = 0, 1
FLOOR_FIXED, FLOOR_DRIFT = 0, 1
BC_OUTFLOW, BC_POLAR, BC_PERIODIC = 0, 1, 2


def build() -> str:
    """Compile orc.c with gcc (-O2, no FMA contraction) into liborc.so."""
    src = os.path.join(_HERE, "orc.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99",
                           "-Wall", "-o", tmp, src, "-lm"])
    os.replace(tmp, _SO)
    return _SO


class Desc(C.Structure):
    _fields_ = [("coords", C.c_int32), ("n", C.c_int32 * 3), ("ng", C.c_int32),
                ("recon", C.c_int32), ("riemann", C.c_int32), ("bc", C.c_int32 * 6),
                ("maxit", C.c_int32), ("guess_mode", C.c_int32),
                ("a", C.c_double), ("gam", C.c_double),
                ("xlo", C.c_double * 3), ("xhi", C.c_double * 3), ("courant", C.c_double),
                ("rho_fl_c", C.c_double), ("rho_fl_p", C.c_double), ("u_fl_c", C.c_double),
                ("u_fl_p", C.c_double), ("bsq_rho_max", C.c_double), ("bsq_u_max", C.c_double),
                ("gamma_max", C.c_double), ("tol", C.c_double), ("emf", C.c_int32),
                ("floor_frame", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("tier", C.c_int64 * 5), ("iter_hist", C.c_int64 * 64),
                ("floor_hits", C.c_int64), ("cells", C.c_int64)]


_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(Desc)]
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_np.restype = C.c_int
        L.orc_np.argtypes = [C.c_void_p, C.c_int]
        L.orc_geom_point.argtypes = [C.POINTER(Desc), C.c_double, C.c_double, _dp, _dp,
                                     C.POINTER(C.c_double), C.POINTER(C.c_double), _dp]
        L.orc_prim_to_flux.argtypes = [_dp, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                       C.c_int, _dp]
        L.orc_vchar.argtypes = [_dp, _dp, _dp, _dp, C.c_double, C.c_double, C.c_int,
                                C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_source.argtypes = [_dp, _dp, _dp, _dp, C.c_double, C.c_double, _dp, C.c_double, _dp]
        L.orc_recon_face.argtypes = [C.c_int, _dp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_recon_face_flat.argtypes = [_dp, C.c_double, C.c_double, C.POINTER(C.c_double),
                                          C.POINTER(C.c_double)]
        L.orc_floors.restype = C.c_int
        L.orc_floors.argtypes = [C.c_int, _dp, _dp, _dp, _dp] + [C.c_double] * 9 + [C.c_int]
        L.orc_flatten.restype = C.c_double
        L.orc_flatten.argtypes = [_dp, _dp, C.c_int]
        L.orc_cons2prim.restype = C.c_int
        L.orc_cons2prim.argtypes = [_dp, _dp, _dp, C.c_double, C.c_double, C.c_double, _dp, _dp,
                                    C.c_double, C.c_int, _dp, C.POINTER(C.c_int)]
        L.orc_c2p_bisect.restype = C.c_int
        L.orc_c2p_bisect.argtypes = [_dp, _dp, _dp, C.c_double, C.c_double, C.c_double, _dp]
        L.orc_fill_bc.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_dt.restype = C.c_double
        L.orc_dt.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_stage.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, C.c_double, _dp, _dp,
                                C.POINTER(Stats)]
        L.orc_step.restype = C.c_double
        L.orc_step.argtypes = [C.c_void_p, _dp, _dp, C.c_int, C.c_double, C.POINTER(Stats)]
        L.orc_divb.restype = C.c_double
        L.orc_divb.argtypes = [C.c_void_p, _dp, C.c_void_p, C.c_void_p]
        L.orc_stage_flux.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_stage_apply.argtypes = [C.c_void_p, _dp, _dp, _dp, C.c_double, _dp, _dp, C.c_void_p]
        L.orc_flux_buffer.restype = C.POINTER(C.c_double)
        L.orc_flux_buffer.argtypes = [C.c_void_p]
        L.orc_emf_buffer.restype = C.POINTER(C.c_double)
        L.orc_emf_buffer.argtypes = [C.c_void_p]
        L.orc_last_flux.restype = C.POINTER(C.c_double)
        L.orc_last_flux.argtypes = [C.c_void_p]
        L.orc_last_emf.restype = C.POINTER(C.c_double)
        L.orc_last_emf.argtypes = [C.c_void_p]
        L.orc_reinvert.restype = C.c_int
        L.orc_reinvert.argtypes = [C.c_void_p, _dp, _dp, _dp, C.c_int, C.c_int, C.c_int, _dp,
                                   C.POINTER(Stats)]
        _lib = L
    return _lib


def make_desc(cfg: dict) -> Desc:
    """Build the C descriptor from a plain dict (keys as in the Desc fields)."""
    d = Desc()
    d.coords = cfg["coords"]
    for k in range(3):
        d.n[k] = cfg["n"][k]
        d.xlo[k] = cfg["xlo"][k]
        d.xhi[k] = cfg["xhi"][k]
    d.ng = cfg["ng"]
    d.recon = cfg["recon"]
    d.riemann = cfg["riemann"]
    for k in range(6):
        d.bc[k] = cfg["bc"][k]
    d.maxit = cfg.get("maxit", 50)
    d.guess_mode = 0
    d.a = cfg.get("a", 0.0)
    d.gam = cfg["gam"]
    d.courant = cfg.get("courant", 0.8)
    d.rho_fl_c = cfg.get("rho_fl_c", 0.0)
    d.rho_fl_p = cfg.get("rho_fl_p", 0.0)
    d.u_fl_c = cfg.get("u_fl_c", 0.0)
    d.u_fl_p = cfg.get("u_fl_p", 0.0)
    d.bsq_rho_max = cfg.get("bsq_rho_max", 1e300)
    d.bsq_u_max = cfg.get("bsq_u_max", 1e300)
    d.gamma_max = cfg.get("gamma_max", 1e150)
    d.tol = cfg.get("tol", 1e-12)
    d.emf = cfg.get("emf", EMF_AVERAGE)
    d.floor_frame = cfg.get("floor_frame", FLOOR_FIXED)
    return d


class Grid:
    """A uniform grid handled by the oracle.  State arrays are numpy arrays of shape
    (5, NP3, NP2, NP1) for primitives and (3, NP3, NP2, NP1) for face fields."""

    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        self.desc = make_desc(cfg)
        self.L = lib()
        self.ptr = self.L.orc_create(C.byref(self.desc))
        self.np = tuple(self.L.orc_np(self.ptr, k) for k in range(3))
        self.stats = Stats()

    def __del__(self):
        try:
            self.L.orc_free(self.ptr)
        except Exception:
            pass

    def shape(self, nvar):
        return (nvar, self.np[2], self.np[1], self.np[0])

    def zeros(self):
        return np.zeros(self.shape(5)), np.zeros(self.shape(3))

    def fill_bc(self, P, B):
        self.L.orc_fill_bc(self.ptr, P, B)

    def dt(self, P, B):
        return self.L.orc_dt(self.ptr, P, B)

    def stage(self, Pn, Bn, Ps, Bs, dts, Pout, Bout):
        self.L.orc_stage(self.ptr, Pn, Bn, Ps, Bs, dts, Pout, Bout, C.byref(self.stats))

    def stage_flux(self, Ps, Bs):
        self.L.orc_stage_flux(self.ptr, Ps, Bs)

    def stage_apply(self, Pn, Bn, Ps, dts, Pout, Bout):
        self.L.orc_stage_apply(self.ptr, Pn, Bn, Ps, dts, Pout, Bout, C.byref(self.stats))

    def flux_view(self):
        """writable view of the flux buffer [3][9][NP3][NP2][NP1]"""
        n = 27 * self.np[0] * self.np[1] * self.np[2]
        p = self.L.orc_flux_buffer(self.ptr)
        return np.ctypeslib.as_array(p, shape=(n,)).reshape(3, 9, self.np[2], self.np[1], self.np[0])

    def emf_view(self):
        """writable view of the EMF buffer [3][NP3][NP2][NP1]"""
        n = 3 * self.np[0] * self.np[1] * self.np[2]
        p = self.L.orc_emf_buffer(self.ptr)
        return np.ctypeslib.as_array(p, shape=(n,)).reshape(3, self.np[2], self.np[1], self.np[0])

    def step(self, P, B, nsteps=1, dt_fixed=0.0):
        return self.L.orc_step(self.ptr, P, B, nsteps, dt_fixed, C.byref(self.stats))

    def divb(self, B, field=None):
        if field is None:
            return self.L.orc_divb(self.ptr, B, None, None)
        return self.L.orc_divb(self.ptr, B, field.ctypes.data_as(C.c_void_p), None)

    def divb_rel(self, B, field=None):
        """(max |div B|, max |div B| / sum_d (|B_+| + |B_-|)/dx_d) over interior cells"""
        rel = C.c_double()
        f = None if field is None else field.ctypes.data_as(C.c_void_p)
        a = self.L.orc_divb(self.ptr, B, f, C.cast(C.byref(rel), C.c_void_p))
        return a, rel.value

    def last_flux(self):
        n = 27 * self.np[0] * self.np[1] * self.np[2]
        p = self.L.orc_last_flux(self.ptr)
        return np.ctypeslib.as_array(p, shape=(n,)).reshape(3, 9, self.np[2], self.np[1],
                                                            self.np[0]).copy()

    def last_emf(self):
        n = 3 * self.np[0] * self.np[1] * self.np[2]
        p = self.L.orc_last_emf(self.ptr)
        return np.ctypeslib.as_array(p, shape=(n,)).reshape(3, self.np[2], self.np[1],
                                                            self.np[0]).copy()

    def reinvert(self, P, Bold, Bnew, K, J, I, dU):
        return self.L.orc_reinvert(self.ptr, P, Bold, Bnew, K, J, I,
                                   np.ascontiguousarray(dU, dtype=float), C.byref(self.stats))

    def interior(self, A):
        g = self.cfg["ng"]
        n = self.cfg["n"]
        return A[:, g:g + n[2], g:g + n[1], g:g + n[0]]


def geom_point(cfg: dict, x1: float, x2: float):
    d = make_desc(cfg)
    gcov = np.zeros(16)
    gcon = np.zeros(16)
    conn = np.zeros(64)
    gdet = C.c_double()
    alpha = C.c_double()
    lib().orc_geom_point(C.byref(d), x1, x2, gcov, gcon, C.byref(gdet), C.byref(alpha), conn)
    return gcov.reshape(4, 4), gcon.reshape(4, 4), gdet.value, alpha.value, conn.reshape(4, 4, 4)


def prim_to_flux(P, Bcon, gcov, gcon, gdet, alpha, gam, dir_):
    out = np.zeros(9)
    lib().orc_prim_to_flux(np.ascontiguousarray(P, dtype=float), np.ascontiguousarray(Bcon, dtype=float),
                           np.ascontiguousarray(gcov, dtype=float).ravel(),
                           np.ascontiguousarray(gcon, dtype=float).ravel(), gdet, alpha, gam, dir_, out)
    return out


def vchar(P, Bcon, gcov, gcon, alpha, gam, dir_):
    vmax = C.c_double()
    vmin = C.c_double()
    lib().orc_vchar(np.ascontiguousarray(P, dtype=float), np.ascontiguousarray(Bcon, dtype=float),
                    np.ascontiguousarray(gcov, dtype=float).ravel(),
                    np.ascontiguousarray(gcon, dtype=float).ravel(), alpha, gam, dir_,
                    C.byref(vmax), C.byref(vmin))
    return vmax.value, vmin.value


def source(P, Bcon, gcov, gcon, gdet, alpha, conn, gam):
    out = np.zeros(9)
    lib().orc_source(np.ascontiguousarray(P, dtype=float), np.ascontiguousarray(Bcon, dtype=float),
                     np.ascontiguousarray(gcov, dtype=float).ravel(),
                     np.ascontiguousarray(gcon, dtype=float).ravel(), gdet, alpha,
                     np.ascontiguousarray(conn, dtype=float).ravel(), gam, out)
    return out


def recon_face(recon, a6):
    l = C.c_double()
    r = C.c_double()
    lib().orc_recon_face(recon, np.ascontiguousarray(a6, dtype=float), C.byref(l), C.byref(r))
    return l.value, r.value


def recon_face_flat(a6, f2, f3):
    l = C.c_double()
    r = C.c_double()
    lib().orc_recon_face_flat(np.ascontiguousarray(a6, dtype=float), f2, f3, C.byref(l), C.byref(r))
    return l.value, r.value


def floors(frame, P, Bcon, gcov, gcon, gdet, alpha, gam, rho_fl, u_fl, bsq_rho_max=50.0,
           bsq_u_max=750.0, gamma_max=50.0, tol=1e-12, maxit=50):
    """one cell's floors as the update applies them; returns (new primitives, limits)"""
    P = np.array(P, dtype=float)
    hits = lib().orc_floors(frame, P, np.ascontiguousarray(Bcon, dtype=float),
                            np.ascontiguousarray(gcov, dtype=float).ravel(),
                            np.ascontiguousarray(gcon, dtype=float).ravel(), gdet, alpha, gam,
                            rho_fl, u_fl, bsq_rho_max, bsq_u_max, gamma_max, tol, maxit)
    return P, hits


def flatten(u, v, c):
    return lib().orc_flatten(np.ascontiguousarray(u, dtype=float), np.ascontiguousarray(v, dtype=float), c)


def cons2prim(U, gcov, gcon, gdet, alpha, gam, guess, prev=None, tol=1e-12, maxit=50):
    P = np.zeros(5)
    it = C.c_int()
    guess = np.ascontiguousarray(guess, dtype=float)
    prev = guess if prev is None else np.ascontiguousarray(prev, dtype=float)
    tier = lib().orc_cons2prim(np.ascontiguousarray(U, dtype=float),
                               np.ascontiguousarray(gcov, dtype=float).ravel(),
                               np.ascontiguousarray(gcon, dtype=float).ravel(), gdet, alpha, gam,
                               guess, prev, tol, maxit, P, C.byref(it))
    return P, tier, it.value


def c2p_bisect(U, gcov, gcon, gdet, alpha, gam):
    P = np.zeros(5)
    rc = lib().orc_c2p_bisect(np.ascontiguousarray(U, dtype=float),
                              np.ascontiguousarray(gcov, dtype=float).ravel(),
                              np.ascontiguousarray(gcon, dtype=float).ravel(), gdet, alpha, gam, P)
    return P, rc
