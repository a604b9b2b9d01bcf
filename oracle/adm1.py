"""ctypes binding of the plain FP64 ADM1 oracle (adm1_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
CPU-baseline leg of the benchmark use it; the HIP product path never does.
It reads the parameter file itself and imports nothing from the product
package.

State arrays are structure-of-arrays ``x[35][ld]`` in float64, the same
layout the product's C ABI uses, so one seeded input serves both sides.
"""
from __future__ import annotations

import ctypes
import json
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "adm1_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
DEFAULT_PARAMS = os.path.join(os.path.dirname(HERE), "paper_2311_08927_amd", "data",
                              "adm1_params.json")

NX, ND, NLIQ, NPROC = 35, 28, 26, 19
# integration order of the 28 differential entries (state indices)
DIFF = [0, 1, 2, 3, 4, 5, 6, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22,
        23, 24, 25, 32, 33, 34]
ALG = [7, 26, 27, 28, 29, 30, 31]
STATUS_NAMES = {0: "ok", 1: "algebraic", 2: "underflow", 3: "max_steps", 4: "nonfinite"}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C11, -O2)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, SRC,
                               "-lm", "-lpthread"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_param_names.restype = ctypes.c_char_p
        L.orc_param_count.restype = ctypes.c_int
        L.orc_params_doubles.restype = ctypes.c_int
        L.orc_check_params.restype = ctypes.c_int
        L.orc_run.restype = ctypes.c_int
        L.orc_run.argtypes = [ctypes.c_void_p, ctypes.c_void_p, dp, ctypes.c_int64, dp, dp,
                              ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_int64,
                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
        L.orc_run_fixed.restype = ctypes.c_int
        L.orc_run_fixed.argtypes = [ctypes.c_void_p, ctypes.c_void_p, dp, ctypes.c_int64, dp,
                                    dp, ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_int, ctypes.c_void_p]
        L.orc_rhs.restype = ctypes.c_int
        L.orc_rhs.argtypes = [ctypes.c_void_p, ctypes.c_void_p, dp, ctypes.c_double,
                              ctypes.c_double, dp, dp, dp, dp, ctypes.c_double]
        L.orc_jacobian.restype = ctypes.c_int
        L.orc_jacobian.argtypes = [ctypes.c_void_p, ctypes.c_void_p, dp, ctypes.c_double,
                                   ctypes.c_double, dp, dp, ctypes.c_double]
        L.orc_solve_ph.restype = ctypes.c_int
        L.orc_solve_ph.argtypes = [ctypes.c_void_p, ctypes.c_void_p, dp, ctypes.c_double,
                                   ctypes.c_double, dp]
        L.orc_solve_h2.restype = ctypes.c_int
        L.orc_solve_h2.argtypes = [ctypes.c_void_p, ctypes.c_void_p, dp, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc_charge_residual.restype = ctypes.c_double
        L.orc_charge_residual.argtypes = [ctypes.c_void_p, dp, ctypes.c_double,
                                          ctypes.c_double]
        L.orc_h2_residual.restype = ctypes.c_double
        L.orc_h2_residual.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double]
        L.orc_rates.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_gas_flux.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_fixed.restype = ctypes.c_int
        L.orc_fixed.argtypes = [ctypes.c_void_p, ctypes.c_void_p, dp, ctypes.c_double,
                                ctypes.c_double, dp, ctypes.c_double, ctypes.c_int,
                                ctypes.c_int, ctypes.c_double]
        L.orc_petersen.argtypes = [ctypes.c_void_p, dp]
        L.orc_contents.argtypes = [ctypes.c_void_p, dp, dp]
        L.orc_inhib.restype = ctypes.c_double
        L.orc_inhib.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double]
        L.orc_tconst_export.argtypes = [ctypes.c_void_p, ctypes.c_double, dp]
        L.orc_rodas4_tableau.argtypes = [dp, dp, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vp(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def particle_kin(phase, phase_kin, n):
    """Per-particle kinetic factors from phase ids and the factor of each id
    (ids beyond the table: 1); None when there are no phases."""
    if phase is None:
        return None
    table = np.ones(256)
    if phase_kin is not None:
        k = np.asarray(phase_kin, dtype=np.float64)
        table[:k.size] = k
    ph = np.asarray(phase)[:n]
    assert ph.dtype == np.uint8
    return np.ascontiguousarray(table[ph])


class Oracle:
    """Parameters + options, and the oracle calls on numpy arrays."""

    def __init__(self, params: dict | str | None = None, rtol: float = 1e-8,
                 atol=None, max_steps: int = 100000, newton_tol: float = 1e-14,
                 newton_maxit: int = 100, model: str | None = None):
        if params is None or isinstance(params, str):
            with open(params or DEFAULT_PARAMS) as fh:
                params = json.load(fh)["values"]
        self.values = dict(params)
        L = lib()
        names = L.orc_param_names().decode().split(",")[:-1]
        assert len(names) == L.orc_param_count()
        size = L.orc_params_doubles()
        assert size == len(names) + NLIQ * NPROC + 2 * NLIQ + 1
        self._p = (ctypes.c_double * size)(*[float(self.values[n]) for n in names])
        self.model = model
        if model is not None:
            # the description's matrix and contents, by the oracle's own reader
            from oracle import model_desc
            nu, C, N = model_desc.tables(model_desc.load(model), self.values)
            base = len(names)
            flat = np.concatenate([nu.ravel(), C, N, [1.0]])
            for k, v in enumerate(flat):
                self._p[base + k] = float(v)
        if L.orc_check_params(ctypes.byref(self._p)) != 0:
            raise ValueError("parameter set violates COD continuity")
        if atol is None:
            atol = np.full(ND, 1e-12)
        atol = np.asarray(atol, dtype=np.float64)
        assert atol.shape == (ND,)

        class _Opts(ctypes.Structure):
            _fields_ = [("rtol", ctypes.c_double), ("atol", ctypes.c_double * ND),
                        ("max_steps", ctypes.c_int), ("newton_tol", ctypes.c_double),
                        ("newton_maxit", ctypes.c_int)]

        self._o = _Opts(rtol, (ctypes.c_double * ND)(*atol), max_steps, newton_tol,
                        newton_maxit)
        self.rtol, self.atol = rtol, atol

    # -- per-particle pieces -------------------------------------------------
    def rhs(self, x, T, D, s_in, H_guess=-1.0, kin=1.0):
        """f (28, integration order), consistent 35-state, S_H+; kin: the
        kinetic factor of the particle's phase."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        s_in = np.ascontiguousarray(s_in, dtype=np.float64)
        f = np.zeros(ND); xa = np.zeros(NX); H = np.array([H_guess])
        rc = lib().orc_rhs(ctypes.byref(self._p), ctypes.byref(self._o), _dp(x), T, D,
                           _dp(s_in), _dp(f), _dp(xa), _dp(H), float(kin))
        if rc != 0:
            raise RuntimeError("algebraic solve failed")
        return f, xa, float(H[0])

    def jacobian(self, x, T, D, s_in, kin=1.0):
        x = np.ascontiguousarray(x, dtype=np.float64)
        s_in = np.ascontiguousarray(s_in, dtype=np.float64)
        J = np.zeros((ND, ND))
        rc = lib().orc_jacobian(ctypes.byref(self._p), ctypes.byref(self._o), _dp(x), T, D,
                                _dp(s_in), _dp(J), float(kin))
        if rc != 0:
            raise RuntimeError("algebraic solve failed")
        return J

    def solve_ph(self, x, T, guess=-1.0):
        x = np.ascontiguousarray(x, dtype=np.float64)
        H = np.zeros(1)
        rc = lib().orc_solve_ph(ctypes.byref(self._p), ctypes.byref(self._o), _dp(x), T,
                                guess, _dp(H))
        if rc != 0:
            raise RuntimeError("eq. 7 solve failed")
        return float(H[0])

    def solve_h2(self, x, T, H, D, s_in_h2):
        x = np.ascontiguousarray(x, dtype=np.float64)
        S = np.zeros(1)
        rc = lib().orc_solve_h2(ctypes.byref(self._p), ctypes.byref(self._o), _dp(x), T, H,
                                D, s_in_h2, _dp(S))
        if rc != 0:
            raise RuntimeError("eq. 8 solve failed")
        return float(S[0])

    def charge_residual(self, x, T, H):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return lib().orc_charge_residual(ctypes.byref(self._p), _dp(x), T, H)

    def h2_residual(self, x, T, H, D, s_in_h2):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return lib().orc_h2_residual(ctypes.byref(self._p), _dp(x), T, H, D, s_in_h2)

    def rates(self, x, T, H):
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.zeros(27)
        lib().orc_rates(ctypes.byref(self._p), _dp(x), T, H, _dp(out))
        return out

    def gas_flux(self, x, T, V_liq):
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.zeros(4)
        lib().orc_gas_flux(ctypes.byref(self._p), _dp(x), T, V_liq, _dp(out))
        return out

    def tconst(self, T):
        out = np.zeros(9)
        lib().orc_tconst_export(ctypes.byref(self._p), T, _dp(out))
        return dict(zip(["RT", "K_w", "K_a_co2", "K_a_IN", "K_H_h2", "K_H_ch4", "K_H_co2",
                         "p_h2o", "arr"], out))

    def petersen(self):
        nu = np.zeros((NLIQ, NPROC))
        lib().orc_petersen(ctypes.byref(self._p), _dp(nu))
        return nu

    def contents(self):
        C = np.zeros(NLIQ); N = np.zeros(NLIQ)
        lib().orc_contents(ctypes.byref(self._p), _dp(C), _dp(N))
        return C, N

    def fixed(self, x, T, D, s_in, dt, nsteps, method="rk4", kin=1.0):
        """nsteps equal steps of `method` over dt: "rk4", "rodas4" (no step
        control) or "euler" (the explicit update of the paper's fixed-step
        scheme, sec. 2.3 and 4.3); then the algebraic write-back."""
        x = np.array(x, dtype=np.float64)
        s_in = np.ascontiguousarray(s_in, dtype=np.float64)
        code = {"rk4": 0, "rodas4": 1, "euler": 2}[method]
        rc = lib().orc_fixed(ctypes.byref(self._p), ctypes.byref(self._o), _dp(x), T, D,
                             _dp(s_in), dt, nsteps, code, float(kin))
        if rc != 0:
            raise RuntimeError("fixed-step integration failed")
        return x

    def run_fixed(self, X, T, D, fidx, feed, dt, nsteps, method="euler", n=None,
                  nthreads=None, phase=None, phase_kin=None):
        """The fixed-step scheme (see `fixed`) over particles 0..n-1 of X[35][ld]
        in place, equal particle chunks over nthreads threads.  Returns status
        uint8[n] (1 where a particle's integration failed)."""
        assert X.dtype == np.float64 and X.flags["C_CONTIGUOUS"] and X.shape[0] == NX
        ld = X.shape[1]
        n = ld if n is None else n
        T = np.ascontiguousarray(T, dtype=np.float64)
        D = np.ascontiguousarray(D, dtype=np.float64)
        fidx = np.ascontiguousarray(fidx, dtype=np.int32)
        feed = np.ascontiguousarray(feed, dtype=np.float64)
        code = {"rk4": 0, "rodas4": 1, "euler": 2}[method]
        status = np.zeros(n, dtype=np.uint8)
        kin = particle_kin(phase, phase_kin, n)     # referenced until the call returns
        if nthreads is None:
            nthreads = len(os.sched_getaffinity(0))
        rc = lib().orc_run_fixed(ctypes.byref(self._p), ctypes.byref(self._o), _dp(X), ld,
                                 _dp(T), _dp(D), _vp(fidx), _dp(feed), dt, int(nsteps), code,
                                 n, _vp(status), int(nthreads), _vp(kin))
        if rc != 0:
            raise RuntimeError("oracle fixed-step run failed")
        return status

    # -- batched step ----------------------------------------------------------
    def step(self, X, T, D, fidx, feed, dt, H=None, hlast=None, nthreads=None,
             n=None, phase=None, phase_kin=None):
        """Advance particles in place.  X: float64 [35][ld].  phase: uint8
        phase id per particle (None: all factor 1); phase_kin: kinetic factor
        per id (ids beyond it: 1).  Returns (status uint8[n], stats
        int32[3][ld]: accepted, rejected, newton)."""
        assert X.dtype == np.float64 and X.flags["C_CONTIGUOUS"] and X.shape[0] == NX
        ld = X.shape[1]
        n = ld if n is None else n
        T = np.ascontiguousarray(T, dtype=np.float64)
        D = np.ascontiguousarray(D, dtype=np.float64)
        fidx = np.ascontiguousarray(fidx, dtype=np.int32)
        feed = np.ascontiguousarray(feed, dtype=np.float64)
        assert feed.ndim == 2 and feed.shape[1] == NLIQ
        status = np.zeros(n, dtype=np.uint8)
        stats = np.zeros((3, ld), dtype=np.int32)
        kin = particle_kin(phase, phase_kin, n)     # referenced until the call returns
        if nthreads is None:
            nthreads = len(os.sched_getaffinity(0))
        rc = lib().orc_run(ctypes.byref(self._p), ctypes.byref(self._o), _dp(X), ld,
                           _dp(T), _dp(D), _vp(fidx), _dp(feed), dt, n, _vp(H), _vp(hlast),
                           _vp(status), _vp(stats), int(nthreads), _vp(kin))
        if rc != 0:
            raise RuntimeError("oracle run failed")
        return status, stats

    def rodas4_tableau(self):
        g = np.zeros(1); A = np.zeros((6, 5)); C = np.zeros((6, 5))
        lib().orc_rodas4_tableau(_dp(g), _dp(A), _dp(C))
        return float(g[0]), A, C
