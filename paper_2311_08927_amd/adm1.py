"""Thin ctypes binding of libadm1.so (the C ABI in include/adm1.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels.  Functions carry the C names; tensors are torch CUDA tensors whose
data pointers are passed through, streams are torch streams (default: the
current stream).  If the library is missing, the first call raises.
"""
from __future__ import annotations

import ctypes
import json
import math
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libadm1.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "adm1.h")
NX, ND, NLIQ = 35, 28, 26

VARIANT_DENSE1, VARIANT_SPARSE1, VARIANT_SPARSE2, VARIANT_SPARSE1_LDS = 0, 1, 2, 3
ERRORS = {0: "ok", -1: "E_NULL", -2: "E_SIZE", -3: "E_NOT_DEVICE", -4: "E_PARAMS",
          -5: "E_OPTS", -6: "E_FEED", -7: "E_NOMEM", -8: "E_VARIANT", -9: "E_DT",
          -10: "E_IO", -11: "E_STATIC"}

_libs: dict = {}     # library path -> loaded library
_owner: dict = {}    # context / graph handle -> the library that created it


class ADM1Error(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {code} ({strerror(code)})")


class adm1_opts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("atol", ctypes.c_double * ND),
                ("max_steps", ctypes.c_int32), ("newton_tol", ctypes.c_double),
                ("newton_maxit", ctypes.c_int32), ("rate_precision", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("pivot_floor", ctypes.c_double)]


class adm1_feed(ctypes.Structure):
    _fields_ = [("D", ctypes.c_void_p), ("idx", ctypes.c_void_p), ("S_in", ctypes.c_void_p),
                ("n_feed", ctypes.c_int64), ("phase", ctypes.c_void_p)]


class adm1_aux(ctypes.Structure):
    _fields_ = [("H", ctypes.c_void_p), ("h_last", ctypes.c_void_p)]


def lib_path(model: str | None = None) -> str:
    """Library of a model description by name: lib<model>.so (None or "adm1":
    libadm1.so, the standard matrix)."""
    if model is None or model == "adm1":
        return LIB_PATH
    return os.path.join(PKG, f"lib{model}.so")


def lib(model: str | None = None):
    """Load the library of a model description (default: the standard ADM1
    matrix, libadm1.so); raises if it has not been built."""
    path = lib_path(model)
    if path not in _libs:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: the HIP extension is not built "
                               "(run __graft_entry__.build())")
        L = ctypes.CDLL(path)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.adm1_param_names.restype = ctypes.c_char_p
        L.adm1_strerror.restype = ctypes.c_char_p
        L.adm1_strerror.argtypes = [ctypes.c_int]
        L.adm1_init.restype = ctypes.c_int
        L.adm1_init.argtypes = [vp, vp, i64, ctypes.POINTER(vp)]
        L.adm1_set_opts.restype = ctypes.c_int
        L.adm1_set_opts.argtypes = [vp, vp]
        L.adm1_destroy.argtypes = [vp]
        L.adm1_step_particles.restype = ctypes.c_int
        L.adm1_step_particles.argtypes = [vp, vp, i64, vp, vp, dbl, i64, vp, vp, vp, vp]
        L.adm1_step_particles_static.restype = ctypes.c_int
        L.adm1_step_particles_static.argtypes = [vp, vp, i64, vp, vp, dbl, i64, vp, vp, vp, vp]
        L.adm1_step_fixed.restype = ctypes.c_int
        L.adm1_step_fixed.argtypes = [vp, vp, i64, vp, vp, dbl, i32, i32, i64, vp, vp, vp, vp]
        L.adm1_gas_flux.restype = ctypes.c_int
        L.adm1_gas_flux.argtypes = [vp, vp, i64, vp, vp, i64, vp, vp, vp, vp]
        L.adm1_rhs.restype = ctypes.c_int
        L.adm1_rhs.argtypes = [vp, vp, i64, vp, vp, i64, vp, i64, vp, i32, vp, vp]
        L.adm1_solve_ph.restype = ctypes.c_int
        L.adm1_solve_ph.argtypes = [vp, vp, i64, vp, i64, vp, vp, vp, vp, vp]
        L.adm1_last_failures.restype = ctypes.c_int
        L.adm1_last_failures.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), vp]
        L.adm1_jacobian.restype = ctypes.c_int
        L.adm1_jacobian.argtypes = [vp, vp, i64, vp, vp, i64, vp, vp, vp]
        L.adm1_set_launch.restype = ctypes.c_int
        L.adm1_set_launch.argtypes = [vp, i32, i32]
        L.adm1_set_service_batch.restype = ctypes.c_int
        L.adm1_set_service_batch.argtypes = [vp, i32]
        L.adm1_set_order.restype = ctypes.c_int
        L.adm1_set_order.argtypes = [vp, i32]
        L.adm1_cost_order.restype = ctypes.c_int
        L.adm1_cost_order.argtypes = [vp, vp, dbl, i64, vp, vp]
        L.adm1_graph_capture_step.restype = ctypes.c_int
        L.adm1_graph_capture_step.argtypes = [vp, vp, i64, vp, vp, dbl, i64, vp, vp, vp, vp,
                                              vp, vp, vp, vp, ctypes.POINTER(vp)]
        L.adm1_graph_launch.restype = ctypes.c_int
        L.adm1_graph_launch.argtypes = [vp, vp]
        L.adm1_graph_destroy.argtypes = [vp]
        L.adm1_advect.restype = ctypes.c_int
        L.adm1_advect.argtypes = [vp, i64, i64, vp, dbl, i32, vp]
        L.adm1_feed_mask.restype = ctypes.c_int
        L.adm1_feed_mask.argtypes = [vp, i64, i64, dbl, dbl, dbl, i32, i32, vp, vp, vp, vp]
        L.adm1_grid_create.restype = ctypes.c_int
        L.adm1_grid_create.argtypes = [vp, i64, ctypes.POINTER(vp)]
        L.adm1_grid_destroy.argtypes = [vp]
        L.adm1_diffuse.restype = ctypes.c_int
        L.adm1_diffuse.argtypes = [vp, vp, i64, vp, i64, dbl, i32, vp, vp]
        L.adm1_model_name.restype = ctypes.c_char_p
        L.adm1_set_phase_kinetics.restype = ctypes.c_int
        L.adm1_set_phase_kinetics.argtypes = [vp, vp, i32]
        want = "adm1" if model is None else model
        got = L.adm1_model_name().decode()
        if got != want:
            raise RuntimeError(f"{path} was generated from model {got!r}, not {want!r}")
        _libs[path] = L
    return _libs[path]


def _L(handle):
    """The library that created a context or graph handle."""
    return _owner.get(handle) or lib()


def model_name(ctx) -> str:
    return _L(ctx).adm1_model_name().decode()


def strerror(code: int) -> str:
    return lib().adm1_strerror(int(code)).decode()


def param_names() -> list[str]:
    return lib().adm1_param_names().decode().split(",")[:-1]


def load_params(path: str | None = None) -> dict:
    path = path or os.path.join(PKG, "data", "adm1_params.json")
    with open(path) as fh:
        return json.load(fh)["values"]


def make_params(values: dict):
    names = param_names()
    arr = (ctypes.c_double * len(names))(*[float(values[n]) for n in names])
    return arr


PIVOT_FLOOR = 1e-8  # default growth guard of the static-order factorisations


def make_opts(rtol=1e-8, atol=None, max_steps=100000, newton_tol=1e-14, newton_maxit=100,
              rate_precision=0, variant=-1, pivot_floor=PIVOT_FLOOR) -> adm1_opts:
    if atol is None:
        atol = np.full(ND, 1e-12)
    atol = np.asarray(atol, dtype=np.float64)
    assert atol.shape == (ND,)
    return adm1_opts(rtol, (ctypes.c_double * ND)(*atol), max_steps, newton_tol, newton_maxit,
                     rate_precision, variant, pivot_floor)


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _check(rc: int, what: str):
    if rc != 0:
        raise ADM1Error(rc, what)


def feed_struct(D, idx, S_in, phase=None) -> adm1_feed:
    return adm1_feed(_ptr(D), _ptr(idx), _ptr(S_in), int(S_in.shape[0]), _ptr(phase))


# ---------------------------------------------------------------------------
# C-named entry points
# ---------------------------------------------------------------------------
def adm1_init(params, opts: adm1_opts, n_max: int, model: str | None = None) -> int:
    """Create a context in the library of `model` (default: the standard
    matrix); returns the opaque handle (int)."""
    if isinstance(params, dict):
        params = make_params(params)
    h = ctypes.c_void_p()
    L = lib(model)
    _check(L.adm1_init(ctypes.byref(params), ctypes.byref(opts), int(n_max),
                       ctypes.byref(h)), "adm1_init")
    _owner[h.value] = L
    return h.value


def adm1_set_opts(ctx: int, opts: adm1_opts):
    _check(_L(ctx).adm1_set_opts(ctx, ctypes.byref(opts)), "adm1_set_opts")


def adm1_destroy(ctx: int):
    _L(ctx).adm1_destroy(ctx)
    _owner.pop(ctx, None)


def adm1_step_particles(ctx, state, ld, temp_K, feed: adm1_feed, dt_days, n, aux=None,
                        status=None, nsteps=None, stream=None, check=True) -> int:
    rc = _L(ctx).adm1_step_particles(ctx, _ptr(state), int(ld), _ptr(temp_K),
                                   ctypes.byref(feed), float(dt_days), int(n),
                                   None if aux is None else ctypes.byref(aux), _ptr(status),
                                   _ptr(nsteps), _stream(stream))
    if check:
        _check(rc, "adm1_step_particles")
    return rc


STATIC_MAX_N = 1048576


def adm1_step_particles_static(ctx, state, ld, temp_K, feed: adm1_feed, dt_days, n, aux=None,
                               status=None, nsteps=None, stream=None, check=True) -> int:
    """adm1_step_particles with the work buffers in the library's static
    device array (no allocation; n <= STATIC_MAX_N)."""
    rc = _L(ctx).adm1_step_particles_static(ctx, _ptr(state), int(ld), _ptr(temp_K),
                                          ctypes.byref(feed), float(dt_days), int(n),
                                          None if aux is None else ctypes.byref(aux),
                                          _ptr(status), _ptr(nsteps), _stream(stream))
    if check:
        _check(rc, "adm1_step_particles_static")
    return rc


FIXED_EULER, FIXED_RK4 = 0, 1


def adm1_step_fixed(ctx, state, ld, temp_K, feed: adm1_feed, dt_days, substeps, method, n,
                    H=None, status=None, newton=None, stream=None, check=True) -> int:
    rc = _L(ctx).adm1_step_fixed(ctx, _ptr(state), int(ld), _ptr(temp_K), ctypes.byref(feed),
                               float(dt_days), int(substeps), int(method), int(n), _ptr(H),
                               _ptr(status), _ptr(newton), _stream(stream))
    if check:
        _check(rc, "adm1_step_fixed")
    return rc


def adm1_gas_flux(ctx, state, ld, temp_K, V_liq, n, q_gas, q_ch4, totals, stream=None,
                  check=True) -> int:
    rc = _L(ctx).adm1_gas_flux(ctx, _ptr(state), int(ld), _ptr(temp_K), _ptr(V_liq), int(n),
                             _ptr(q_gas), _ptr(q_ch4), _ptr(totals), _stream(stream))
    if check:
        _check(rc, "adm1_gas_flux")
    return rc


def adm1_rhs(ctx, state, ld, temp_K, feed: adm1_feed, n, dxdt, ld_out, H_out=None,
             rate_precision=0, status=None, stream=None, check=True) -> int:
    rc = _L(ctx).adm1_rhs(ctx, _ptr(state), int(ld), _ptr(temp_K), ctypes.byref(feed), int(n),
                        _ptr(dxdt), int(ld_out), _ptr(H_out), int(rate_precision),
                        _ptr(status), _stream(stream))
    if check:
        _check(rc, "adm1_rhs")
    return rc


def adm1_solve_ph(ctx, state, ld, temp_K, n, H_guess, H_out, pH_out=None, status=None,
                  stream=None, check=True) -> int:
    rc = _L(ctx).adm1_solve_ph(ctx, _ptr(state), int(ld), _ptr(temp_K), int(n), _ptr(H_guess),
                             _ptr(H_out), _ptr(pH_out), _ptr(status), _stream(stream))
    if check:
        _check(rc, "adm1_solve_ph")
    return rc


FAIL_SLOTS = 7
FAIL_NAMES = ["failed", "algebraic", "underflow", "max_steps", "nonfinite", "negative",
              "counted"]


def adm1_last_failures(ctx, stream=None) -> dict:
    """Outcome counts of the last step call (synchronous)."""
    out = (ctypes.c_int64 * FAIL_SLOTS)()
    _check(_L(ctx).adm1_last_failures(ctx, out, _stream(stream)), "adm1_last_failures")
    return dict(zip(FAIL_NAMES, [int(v) for v in out]))


def adm1_jacobian(ctx, state, ld, temp_K, feed: adm1_feed, n, J, status=None, stream=None,
                  check=True) -> int:
    rc = _L(ctx).adm1_jacobian(ctx, _ptr(state), int(ld), _ptr(temp_K), ctypes.byref(feed),
                             int(n), _ptr(J), _ptr(status), _stream(stream))
    if check:
        _check(rc, "adm1_jacobian")
    return rc


FLOW_MODES = 8


class adm1_flow(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("R", ctypes.c_double), ("H", ctypes.c_double),
                ("a", ctypes.c_double * FLOW_MODES), ("nmodes", ctypes.c_int32)]


def make_flow(d: dict) -> adm1_flow:
    a = list(d["a"])
    return adm1_flow(d["omega"], d["R"], d["H"],
                     (ctypes.c_double * FLOW_MODES)(*(a + [0.0] * (FLOW_MODES - len(a)))),
                     len(a))


class adm1_diffusion(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("D", ctypes.c_double), ("V_p", ctypes.c_double),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3)]


def make_diffusion(h, D, V_p, lo, hi) -> adm1_diffusion:
    return adm1_diffusion(float(h), float(D), float(V_p), (ctypes.c_double * 3)(*lo),
                          (ctypes.c_double * 3)(*hi))


def adm1_grid_create(d: adm1_diffusion, n_max: int, check=True):
    out = ctypes.c_void_p()
    rc = lib().adm1_grid_create(ctypes.byref(d), int(n_max), ctypes.byref(out))
    if check:
        _check(rc, "adm1_grid_create")
    return out.value if rc == 0 else rc


def adm1_grid_destroy(g):
    lib().adm1_grid_destroy(g)


def adm1_diffuse(g, state, ld, pos, n, dt_days, substeps, neighbours=None, stream=None,
                 check=True) -> int:
    rc = lib().adm1_diffuse(g, _ptr(state), int(ld), _ptr(pos), int(n), float(dt_days),
                            int(substeps), _ptr(neighbours), _stream(stream))
    if check:
        _check(rc, "adm1_diffuse")
    return rc


class Grid:
    """Owner of an adm1_grid (the neighbour grid of adm1_diffuse)."""

    def __init__(self, d: adm1_diffusion, n_max: int):
        self.handle = adm1_grid_create(d, n_max)
        self.h, self.D = d.h, d.D

    def stable_substeps(self, dt_days: float) -> int:
        """Explicit substeps for dt_days with each at most 0.05 h^2 / D: the
        operator's rates reach about 28 D / h^2 for randomly placed particles
        (Gershgorin, with row sums up to twice the even-spread 3.5 / h^2),
        and explicit Euler needs substep x rate <= 2."""
        if self.D <= 0.0:
            return 1
        return max(1, int(math.ceil(dt_days * self.D / (0.05 * self.h * self.h))))

    def diffuse(self, state, pos, n, dt_days, substeps=1, neighbours=None, stream=None):
        adm1_diffuse(self.handle, state, state.shape[1], pos, n, dt_days, substeps, neighbours,
                     stream)

    def close(self):
        if getattr(self, "handle", None):
            adm1_grid_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def adm1_advect(pos, ld, n, flow: adm1_flow, dt_seconds, substeps, stream=None):
    _check(lib().adm1_advect(_ptr(pos), int(ld), int(n), ctypes.byref(flow),
                             float(dt_seconds), int(substeps), _stream(stream)), "adm1_advect")


def adm1_feed_mask(pos, ld, n, z_min, r_max, D_zone, fidx_zone, fidx_out, D, fidx, flag=None,
                   stream=None):
    _check(lib().adm1_feed_mask(_ptr(pos), int(ld), int(n), float(z_min), float(r_max),
                                float(D_zone), int(fidx_zone), int(fidx_out), _ptr(D),
                                _ptr(fidx), _ptr(flag), _stream(stream)), "adm1_feed_mask")


def adm1_set_launch(ctx: int, variant: int, blocks_per_cu: int = 0):
    _check(_L(ctx).adm1_set_launch(ctx, int(variant), int(blocks_per_cu)), "adm1_set_launch")


ORDER_INDEX, ORDER_COST = 0, 1


MAX_PHASES = 256


def adm1_set_phase_kinetics(ctx: int, kin):
    """Kinetic factor of phase ids 0..len(kin)-1 (host values; every other id
    gets 1)."""
    k = np.ascontiguousarray(kin, dtype=np.float64).ravel()
    _check(_L(ctx).adm1_set_phase_kinetics(ctx, k.ctypes.data if k.size else None,
                                           int(k.size)), "adm1_set_phase_kinetics")


def adm1_set_service_batch(ctx: int, pairs: int):
    _check(_L(ctx).adm1_set_service_batch(ctx, int(pairs)), "adm1_set_service_batch")


def adm1_set_order(ctx: int, mode: int):
    _check(_L(ctx).adm1_set_order(ctx, int(mode)), "adm1_set_order")


def adm1_cost_order(ctx: int, h_last, dt_days, n, order, stream=None):
    _check(_L(ctx).adm1_cost_order(ctx, _ptr(h_last), float(dt_days), int(n), _ptr(order),
                                 _stream(stream)), "adm1_cost_order")


def adm1_graph_capture_step(ctx, state, ld, temp_K, feed: adm1_feed, dt_days, n, aux, status,
                            nsteps, V_liq, q_gas, q_ch4, totals, stream) -> int:
    g = ctypes.c_void_p()
    _check(_L(ctx).adm1_graph_capture_step(
        ctx, _ptr(state), int(ld), _ptr(temp_K), ctypes.byref(feed), float(dt_days), int(n),
        None if aux is None else ctypes.byref(aux), _ptr(status), _ptr(nsteps), _ptr(V_liq),
        _ptr(q_gas), _ptr(q_ch4), _ptr(totals), _stream(stream), ctypes.byref(g)),
        "adm1_graph_capture_step")
    _owner[g.value] = _L(ctx)
    return g.value


def adm1_graph_launch(g: int, stream=None):
    _check(_L(g).adm1_graph_launch(g, _stream(stream)), "adm1_graph_launch")


def adm1_graph_destroy(g: int):
    _L(g).adm1_graph_destroy(g)
    _owner.pop(g, None)


# ---------------------------------------------------------------------------
# Convenience wrapper: a context plus device copies of one workload
# ---------------------------------------------------------------------------
class Context:
    """Owns an adm1 context; methods take torch CUDA tensors."""

    def __init__(self, n_max: int, rtol: float = 1e-8, atol=None, params=None,
                 model: str | None = None, **opt_kw):
        self.values = params if isinstance(params, dict) else load_params(params)
        self.opts = make_opts(rtol=rtol, atol=atol, **opt_kw)
        self.handle = adm1_init(make_params(self.values), self.opts, n_max, model=model)
        self.n_max = n_max
        self.model = model_name(self.handle)

    def set_opts(self, **kw):
        cur = dict(rtol=self.opts.rtol, atol=np.array(self.opts.atol),
                   max_steps=self.opts.max_steps, newton_tol=self.opts.newton_tol,
                   newton_maxit=self.opts.newton_maxit,
                   rate_precision=self.opts.rate_precision, variant=self.opts.variant,
                   pivot_floor=self.opts.pivot_floor)
        cur.update(kw)
        self.opts = make_opts(**cur)
        adm1_set_opts(self.handle, self.opts)

    def close(self):
        if self.handle:
            adm1_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_phase_kinetics(self, kin):
        adm1_set_phase_kinetics(self.handle, kin)

    def step(self, state, T, D, fidx, S_in, dt, n=None, H=None, hlast=None, status=None,
             nsteps=None, stream=None, phase=None):
        import torch
        n = state.shape[1] if n is None else n
        if status is None:
            status = torch.empty(n, dtype=torch.uint8, device=state.device)
        feed = feed_struct(D, fidx, S_in, phase)
        aux = None if H is None and hlast is None else adm1_aux(_ptr(H), _ptr(hlast))
        adm1_step_particles(self.handle, state, state.shape[1], T, feed, dt, n, aux, status,
                            nsteps, stream)
        return status

    def step_fixed(self, state, T, D, fidx, S_in, dt, substeps, method=FIXED_EULER, n=None,
                   H=None, status=None, newton=None, stream=None, phase=None):
        """The fixed-step explicit scheme (adm1_step_fixed) in place."""
        import torch
        n = state.shape[1] if n is None else n
        if status is None:
            status = torch.empty(n, dtype=torch.uint8, device=state.device)
        adm1_step_fixed(self.handle, state, state.shape[1], T,
                        feed_struct(D, fidx, S_in, phase), dt, substeps, method, n, H, status,
                        newton, stream)
        return status

    def rhs(self, state, T, D, fidx, S_in, n=None, rate_precision=0, stream=None, phase=None):
        import torch
        n = state.shape[1] if n is None else n
        ld = state.shape[1]
        dxdt = torch.empty((ND, ld), dtype=torch.float64, device=state.device)
        H = torch.empty(n, dtype=torch.float64, device=state.device)
        st = torch.empty(n, dtype=torch.uint8, device=state.device)
        adm1_rhs(self.handle, state, ld, T, feed_struct(D, fidx, S_in, phase), n, dxdt, ld, H,
                 rate_precision, st, stream)
        return dxdt, H, st

    def solve_ph(self, state, T, n=None, H_guess=None, stream=None):
        """Eq. 7 alone: (S_H+, pH, status) of each particle's totals."""
        import torch
        n = state.shape[1] if n is None else n
        H = torch.empty(n, dtype=torch.float64, device=state.device)
        pH = torch.empty(n, dtype=torch.float64, device=state.device)
        st = torch.empty(n, dtype=torch.uint8, device=state.device)
        adm1_solve_ph(self.handle, state, state.shape[1], T, n, H_guess, H, pH, st, stream)
        return H, pH, st

    def last_failures(self, stream=None) -> dict:
        return adm1_last_failures(self.handle, stream)

    def jacobian(self, state, T, D, fidx, S_in, n=None, stream=None, phase=None):
        import torch
        n = state.shape[1] if n is None else n
        J = torch.empty((n, ND, ND), dtype=torch.float64, device=state.device)
        st = torch.empty(n, dtype=torch.uint8, device=state.device)
        adm1_jacobian(self.handle, state, state.shape[1], T,
                      feed_struct(D, fidx, S_in, phase), n, J, st, stream)
        return J, st

    def gas_flux(self, state, T, V_liq=None, n=None, stream=None):
        import torch
        n = state.shape[1] if n is None else n
        q = torch.empty(n, dtype=torch.float64, device=state.device)
        qc = torch.empty(n, dtype=torch.float64, device=state.device)
        tot = torch.empty(4, dtype=torch.float64, device=state.device)
        adm1_gas_flux(self.handle, state, state.shape[1], T, V_liq, n, q, qc, tot, stream)
        return q, qc, tot
