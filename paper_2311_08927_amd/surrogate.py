"""ctypes binding of the learned-surrogate entry points of libadm1.so and the
host-side training driver.

Argument marshalling only: featurisation, the network, its loss, backward
pass and optimiser, the gate and the fallback integration all run in the
HIP kernels.  The training driver here only orchestrates: it runs the FP64
integrator to produce transitions, asks the kernels for raw features and
targets to take their mean and spread, shuffles batch indices and calls the
training step.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import adm1 as A
from . import workloads as W

IN, HID, OUT = 38, 256, 35
NPARAMS = 216355
FEAT_LD, OUT_LD = 64, 48

_ready = False


class adm1_mlp_norm(ctypes.Structure):
    _fields_ = [("in_mean", ctypes.c_float * IN), ("in_sd", ctypes.c_float * IN),
                ("out_mean", ctypes.c_float * OUT), ("out_sd", ctypes.c_float * OUT),
                ("floor", ctypes.c_double * OUT)]


class adm1_gate(ctypes.Structure):
    _fields_ = [("max_dlog", ctypes.c_double), ("tol_ion", ctypes.c_double),
                ("tol_closure", ctypes.c_double)]


def _lib():
    global _ready
    L = A.lib()
    if not _ready:
        vp, i64, i32, dbl, flt = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                  ctypes.c_double, ctypes.c_float)
        sig = {
            "adm1_surrogate_create": [vp, i64, i64, ctypes.POINTER(vp)],
            "adm1_surrogate_set_weights": [vp, vp, vp],
            "adm1_surrogate_get_weights": [vp, vp, vp],
            "adm1_surrogate_get_grads": [vp, vp],
            "adm1_surrogate_featurize": [vp, vp, i64, vp, vp, dbl, i64, vp, vp],
            "adm1_surrogate_targets": [vp, vp, vp, i64, i64, vp, vp],
            "adm1_surrogate_forward": [vp, vp, i64, vp, vp],
            "adm1_surrogate_gate": [vp, vp, i64, vp, vp, dbl, i64, vp, vp, vp, vp, vp, vp, vp,
                                    vp, vp],
            "adm1_surrogate_step": [vp, vp, i64, vp, vp, dbl, i64, vp, vp, vp, vp, vp, vp, vp],
            "adm1_surrogate_train_step": [vp, vp, vp, i64, flt, i32, vp, vp],
            "adm1_surrogate_residual_stats": [vp, vp, vp, i64, i64, vp, vp, vp],
            "adm1_gather_rows": [vp, i64, i64, vp, i64, vp, vp],
            "adm1_permutation": [i64, ctypes.c_uint64, vp, vp],
            "adm1_column_stats": [vp, i32, i64, i32, i64, vp, vp, vp],
            "adm1_surrogate_graph_capture_step": [vp, vp, i64, vp, vp, dbl, i64, vp, vp, vp,
                                                  vp, vp, vp, vp, vp, vp, vp, vp,
                                                  ctypes.POINTER(vp)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.restype = ctypes.c_int
            f.argtypes = args
        L.adm1_surrogate_destroy.argtypes = [vp]
        L.adm1_surrogate_destroy.restype = None
        _ready = True
    return L


_p, _s, _check = A._ptr, A._stream, A._check


def make_norm(in_mean, in_sd, out_mean, out_sd, floor) -> adm1_mlp_norm:
    f = lambda a, n: (ctypes.c_float * n)(*np.asarray(a, np.float32).tolist())  # noqa: E731
    return adm1_mlp_norm(f(in_mean, IN), f(in_sd, IN), f(out_mean, OUT), f(out_sd, OUT),
                         (ctypes.c_double * OUT)(*np.asarray(floor, np.float64).tolist()))


def norm_dict(n: adm1_mlp_norm) -> dict:
    return {k: np.array(getattr(n, k)) for k in ("in_mean", "in_sd", "out_mean", "out_sd",
                                                 "floor")}


def identity_norm(floor) -> adm1_mlp_norm:
    return make_norm(np.zeros(IN), np.ones(IN), np.zeros(OUT), np.ones(OUT), floor)


def init_params(seed: int) -> np.ndarray:
    """Initial weights: W ~ N(0, 1/fan_in) per layer, zero biases (seeded);
    flat float32 vector in the ABI's layer order."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in ((IN, HID), (HID, HID), (HID, HID), (HID, HID), (HID, OUT)):
        parts += [(rng.standard_normal((i, o)) / math.sqrt(i)).ravel(), np.zeros(o)]
    return np.concatenate(parts).astype(np.float32)


def default_floor() -> np.ndarray:
    """Per-entry floor of the log features: 1e-6 of the nominal state."""
    return 1e-6 * W.nominal()["state"]


# ---------------------------------------------------------------------------
# C-named entry points
# ---------------------------------------------------------------------------
def adm1_surrogate_create(ctx: int, n_max: int, batch_max: int) -> int:
    if A.model_name(ctx) != "adm1":
        # features, targets and the fallback belong to the standard matrix
        raise ValueError(f"the surrogate models the standard ADM1 matrix, not "
                         f"{A.model_name(ctx)!r}")
    h = ctypes.c_void_p()
    _check(_lib().adm1_surrogate_create(ctx, int(n_max), int(batch_max), ctypes.byref(h)),
           "adm1_surrogate_create")
    return h.value


def adm1_surrogate_destroy(s: int):
    _lib().adm1_surrogate_destroy(s)


def adm1_surrogate_set_weights(s: int, params: np.ndarray, norm: adm1_mlp_norm):
    params = np.ascontiguousarray(params, dtype=np.float32)
    assert params.size == NPARAMS
    _check(_lib().adm1_surrogate_set_weights(s, params.ctypes.data, ctypes.byref(norm)),
           "adm1_surrogate_set_weights")


def adm1_surrogate_get_weights(s: int):
    params = np.empty(NPARAMS, dtype=np.float32)
    norm = adm1_mlp_norm()
    _check(_lib().adm1_surrogate_get_weights(s, params.ctypes.data, ctypes.byref(norm)),
           "adm1_surrogate_get_weights")
    return params, norm


def adm1_surrogate_get_grads(s: int) -> np.ndarray:
    g = np.empty(NPARAMS, dtype=np.float32)
    _check(_lib().adm1_surrogate_get_grads(s, g.ctypes.data), "adm1_surrogate_get_grads")
    return g


def adm1_surrogate_featurize(s, state, ld, temp_K, D, dt_days, n, X, stream=None):
    _check(_lib().adm1_surrogate_featurize(s, _p(state), int(ld), _p(temp_K), _p(D),
                                           float(dt_days), int(n), _p(X), _s(stream)),
           "adm1_surrogate_featurize")


def adm1_surrogate_targets(s, x0, x1, ld, n, target, stream=None):
    _check(_lib().adm1_surrogate_targets(s, _p(x0), _p(x1), int(ld), int(n), _p(target),
                                         _s(stream)), "adm1_surrogate_targets")


def adm1_surrogate_forward(s, X, n, Y, stream=None):
    _check(_lib().adm1_surrogate_forward(s, _p(X), int(n), _p(Y), _s(stream)),
           "adm1_surrogate_forward")


def adm1_surrogate_gate(s, state, ld, temp_K, feed, dt_days, n, Y, gate: adm1_gate, aux,
                        status, nsteps, route, fb_idx, fb_count, stream=None):
    _check(_lib().adm1_surrogate_gate(
        s, _p(state), int(ld), _p(temp_K), ctypes.byref(feed), float(dt_days), int(n), _p(Y),
        ctypes.byref(gate), None if aux is None else ctypes.byref(aux), _p(status),
        _p(nsteps), _p(route), _p(fb_idx), _p(fb_count), _s(stream)), "adm1_surrogate_gate")


def adm1_surrogate_step(s, state, ld, temp_K, feed, dt_days, n, gate: adm1_gate, aux, status,
                        nsteps=None, route=None, fb_count=None, stream=None):
    _check(_lib().adm1_surrogate_step(
        s, _p(state), int(ld), _p(temp_K), ctypes.byref(feed), float(dt_days), int(n),
        ctypes.byref(gate), None if aux is None else ctypes.byref(aux), _p(status),
        _p(nsteps), _p(route), _p(fb_count), _s(stream)), "adm1_surrogate_step")


def adm1_surrogate_graph_capture_step(s, state, ld, temp_K, feed, dt_days, n, gate: adm1_gate,
                                      aux, status, nsteps, route, fb_count, V_liq, q_gas,
                                      q_ch4, totals, stream) -> int:
    """Capture the gated step + gas flux as a graph (launch/destroy with
    adm1.adm1_graph_launch / adm1.adm1_graph_destroy)."""
    g = ctypes.c_void_p()
    _check(_lib().adm1_surrogate_graph_capture_step(
        s, _p(state), int(ld), _p(temp_K), ctypes.byref(feed), float(dt_days), int(n),
        ctypes.byref(gate), None if aux is None else ctypes.byref(aux), _p(status), _p(nsteps),
        _p(route), _p(fb_count), _p(V_liq), _p(q_gas), _p(q_ch4), _p(totals), _s(stream),
        ctypes.byref(g)), "adm1_surrogate_graph_capture_step")
    return g.value


def adm1_gather_rows(src, idx, dst, stream=None):
    """dst[j] = src[idx[j]] over rows (device tensors; rows of 4-byte words)."""
    rb = src.stride(0) * src.element_size()
    assert src.is_contiguous() and dst.is_contiguous() and dst.stride(0) * dst.element_size() == rb
    _check(_lib().adm1_gather_rows(_p(src), int(src.shape[0]), int(rb), _p(idx),
                                   int(idx.shape[0]), _p(dst), _s(stream)), "adm1_gather_rows")


def adm1_permutation(n: int, seed: int, out, stream=None):
    _check(_lib().adm1_permutation(int(n), int(seed) & (2**64 - 1), _p(out), _s(stream)),
           "adm1_permutation")


def adm1_column_stats(data, cols: int, bf16: bool, stream=None):
    """(mean, sd) float64 of the first `cols` columns of a 2-D device tensor
    (float32, or BF16 bit patterns in int16 with bf16=True)."""
    mean = np.zeros(cols)
    sd = np.zeros(cols)
    _check(_lib().adm1_column_stats(_p(data), int(bool(bf16)), int(data.shape[0]), int(cols),
                                    int(data.stride(0)), mean.ctypes.data, sd.ctypes.data,
                                    _s(stream)), "adm1_column_stats")
    return mean, sd


def adm1_surrogate_residual_stats(s, X, target, chunk: int = 1 << 20, stream=None):
    """(mean, mean square) float64 [35] of the network's residual on (X, target)."""
    mean = np.zeros(OUT)
    msq = np.zeros(OUT)
    _check(_lib().adm1_surrogate_residual_stats(s, _p(X), _p(target), int(X.shape[0]),
                                                int(chunk), mean.ctypes.data, msq.ctypes.data,
                                                _s(stream)), "adm1_surrogate_residual_stats")
    return mean, msq


def adm1_surrogate_train_step(s, X, target, B, lr, step, loss, stream=None):
    _check(_lib().adm1_surrogate_train_step(s, _p(X), _p(target), int(B), float(lr), int(step),
                                            _p(loss), _s(stream)),
           "adm1_surrogate_train_step")


# ---------------------------------------------------------------------------
# Wrapper and training driver
# ---------------------------------------------------------------------------
class Surrogate:
    """A surrogate bound to a Context (paper_2311_08927_amd.adm1.Context)."""

    def __init__(self, ctx, n_max: int, batch_max: int = 8192):
        self.ctx = ctx
        self.handle = adm1_surrogate_create(ctx.handle, n_max, batch_max)
        self.n_max, self.batch_max = n_max, batch_max
        self.norm = None

    def close(self):
        if self.handle:
            adm1_surrogate_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, params, norm: adm1_mlp_norm):
        adm1_surrogate_set_weights(self.handle, params, norm)
        self.norm = norm

    def get_weights(self):
        return adm1_surrogate_get_weights(self.handle)

    def featurize(self, state, T, D, dt, n=None):
        import torch
        n = state.shape[1] if n is None else n
        X = torch.empty((max(n, 1), FEAT_LD), dtype=torch.int16, device=state.device)
        adm1_surrogate_featurize(self.handle, state, state.shape[1], T, D, dt, n, X)
        return X[:n]

    def targets(self, x0, x1, n=None):
        import torch
        n = x0.shape[1] if n is None else n
        Tg = torch.empty((max(n, 1), OUT), dtype=torch.float32, device=x0.device)
        adm1_surrogate_targets(self.handle, x0, x1, x0.shape[1], n, Tg)
        return Tg[:n]

    def forward(self, X):
        import torch
        n = X.shape[0]
        Y = torch.empty((max(n, 1), OUT_LD), dtype=torch.float32, device=X.device)
        adm1_surrogate_forward(self.handle, X, n, Y)
        return Y[:n]

    def step(self, state, T, D, fidx, S_in, dt, gate: adm1_gate, n=None, H=None, hlast=None,
             status=None, nsteps=None, route=None, fb_count=None, stream=None, phase=None):
        """One gated step (phase: passed through; the library refuses phases
        here, since the surrogate models one phase)."""
        import torch
        n = state.shape[1] if n is None else n
        if status is None:
            status = torch.empty(max(n, 1), dtype=torch.uint8, device=state.device)
        aux = None if H is None and hlast is None else A.adm1_aux(_p(H), _p(hlast))
        adm1_surrogate_step(self.handle, state, state.shape[1], T,
                            A.feed_struct(D, fidx, S_in, phase), dt, n, gate, aux, status,
                            nsteps, route, fb_count, stream)
        return status

    def train_step(self, X, target, lr, step, loss):
        adm1_surrogate_train_step(self.handle, X, target, X.shape[0], lr, step, loss)


def integrate_states(ctx, w: W.Workload, steps: int):
    """Advance w with the FP64 integrator for `steps` coupling intervals.
    Returns the device states X_0..X_steps ([35][ld] each), the dilution
    rates of each interval and a host mask [steps][n] of clean steps
    (status 0)."""
    import torch
    dev = "cuda"
    X = torch.from_numpy(np.ascontiguousarray(w.X)).to(dev)
    T = torch.from_numpy(w.T).to(dev)
    fidx = torch.from_numpy(w.fidx).to(dev)
    S_in = torch.from_numpy(w.feed).to(dev)
    H = torch.full((w.n,), -1.0, dtype=torch.float64, device=dev)
    hl = torch.full((w.n,), -1.0, dtype=torch.float64, device=dev)
    status = torch.empty(w.n, dtype=torch.uint8, device=dev)
    states, Ds, ok = [X.clone()], [], []
    for s in range(steps):
        D = torch.from_numpy(w.D_at(s)).to(dev)
        ctx.step(X, T, D, fidx, S_in, w.dt, n=w.n, H=H, hlast=hl, status=status)
        states.append(X.clone())
        Ds.append(D)
        ok.append(status.cpu().numpy()[:w.n] == 0)
    return states, Ds, np.stack(ok), T


def integrate_field_states(ctx, w: W.Workload, steps: int):
    """Advance a digester field w (workloads.digester_field) with the FP64
    integrator for `steps` coupling intervals, as the coupling driver does:
    feed mask from the positions, step, advection by the seeded flow.
    Returns what integrate_states returns."""
    import torch
    from . import adm1 as A
    dev = "cuda"
    X = torch.from_numpy(np.ascontiguousarray(w.X)).to(dev)
    T = torch.from_numpy(w.T).to(dev)
    S_in = torch.from_numpy(w.feed).to(dev)
    pos = torch.from_numpy(np.ascontiguousarray(w.extra["pos"])).to(dev)
    flow = A.make_flow(w.extra["flow"])
    H = torch.full((w.n,), -1.0, dtype=torch.float64, device=dev)
    hl = torch.full((w.n,), -1.0, dtype=torch.float64, device=dev)
    status = torch.empty(w.n, dtype=torch.uint8, device=dev)
    fidx = torch.empty(w.n, dtype=torch.int32, device=dev)
    dt_s = w.dt * 86400.0
    states, Ds, ok = [X.clone()], [], []
    for s in range(steps):
        D = torch.empty(w.n, dtype=torch.float64, device=dev)
        A.adm1_feed_mask(pos, w.ld, w.n, W.INLET_Z, W.INLET_R, 1.0, 1, 0, D, fidx)
        ctx.step(X, T, D, fidx, S_in, w.dt, n=w.n, H=H, hlast=hl, status=status)
        A.adm1_advect(pos, w.ld, w.n, flow, dt_s, W.advect_substeps(dt_s))
        states.append(X.clone())
        Ds.append(D)
        ok.append(status.cpu().numpy()[:w.n] == 0)
    return states, Ds, np.stack(ok), T


def dataset(sur: "Surrogate", states, Ds, T, dt, n, rows=None):
    """Features and targets (kernel outputs under the surrogate's current
    normalisation) of every transition, stacked step by step; `rows`
    (optional index tensor) selects particles."""
    import torch
    feats, targs = [], []
    for s in range(len(Ds)):
        x0, x1 = states[s], states[s + 1]
        Xs = sur.featurize(x0, T, Ds[s], dt, n)
        Ts = sur.targets(x0, x1, n)
        if rows is not None:
            xr = torch.empty((rows.shape[0], Xs.shape[1]), dtype=Xs.dtype, device=Xs.device)
            tr = torch.empty((rows.shape[0], Ts.shape[1]), dtype=Ts.dtype, device=Ts.device)
            adm1_gather_rows(Xs, rows, xr)
            adm1_gather_rows(Ts, rows, tr)
            Xs, Ts = xr, tr
        feats.append(Xs.clone())
        targs.append(Ts.clone())
    return torch.cat(feats), torch.cat(targs)


def fit_norm(sur: "Surrogate", states, Ds, T, dt, n, floor, rows=None,
             out_weight=None) -> adm1_mlp_norm:
    """Normalisation from the raw (identity-normalised) features and targets
    of the training transitions: per-column mean and spread; columns without
    spread keep unit scale.  out_weight (optional, per output) divides an
    output's spread by its square root, which weights that output's share of
    the mean-squared training loss by out_weight."""
    params, _ = sur.get_weights()
    sur.set_weights(params, identity_norm(floor))
    Xr, Tr = dataset(sur, states, Ds, T, dt, n, rows)
    # BF16-rounded features, as the network sees them; FP64 sums on the device
    in_mean, in_sd = adm1_column_stats(Xr, IN, bf16=True)
    in_sd = np.where(in_sd > 1e-6, in_sd, 1.0)
    out_mean, out_sd = adm1_column_stats(Tr, OUT, bf16=False)
    out_sd = np.where(out_sd > 1e-8, out_sd, 1.0)
    if out_weight is not None:
        out_sd = out_sd / np.sqrt(np.asarray(out_weight, dtype=np.float64))
    return make_norm(in_mean, in_sd, out_mean, out_sd, floor)


def calibrate_output_bias(sur: Surrogate, X, Tg, chunk: int = 1 << 20) -> np.ndarray:
    """Shift the output layer's biases by minus the network's mean residual
    (standardised units) on held-out rows (X, Tg): a coherent bias of the
    predicted increments adds up over a tank of particles and over coupling
    steps, while per-particle scatter averages out.  Returns the shift."""
    shift, _ = adm1_surrogate_residual_stats(sur.handle, X, Tg, chunk)
    params, norm = sur.get_weights()
    params[-OUT:] -= shift.astype(np.float32)
    sur.set_weights(params, norm)
    return -shift


def train(sur: Surrogate, X, Tg, epochs: int, batch: int = 8192, lr: float = 1e-3,
          seed: int = 4, log=None):
    """Adam on (X, Tg) (device tensors, already standardised) with a cosine
    learning-rate schedule; returns the per-epoch mean losses."""
    import torch
    n = X.shape[0]
    nb = n // batch
    total = max(1, epochs * nb)
    loss = torch.zeros(max(nb, 1), dtype=torch.float32, device=X.device)
    perm = torch.empty(n, dtype=torch.int32, device=X.device)
    xb = torch.empty((batch, X.shape[1]), dtype=X.dtype, device=X.device)
    tb = torch.empty((batch, Tg.shape[1]), dtype=Tg.dtype, device=Tg.device)
    hist = []
    k = 0
    for e in range(epochs):
        # a seeded permutation of the rows per epoch, batches gathered on the device
        adm1_permutation(n, (seed << 32) + e, perm)
        for b in range(nb):
            idx = perm[b * batch:(b + 1) * batch]
            adm1_gather_rows(X, idx, xb)
            adm1_gather_rows(Tg, idx, tb)
            k += 1
            lr_k = 0.5 * lr * (1.0 + math.cos(math.pi * (k - 1) / total))
            sur.train_step(xb, tb, lr_k, k, loss[b:b + 1])
        hist.append(float(loss[:nb].cpu().numpy().astype(np.float64).mean()))
        if log:
            log(f"epoch {e}: loss {hist[-1]:.4e}")
    return hist


def train_on_transitions(ctx, sur: Surrogate, train_data: str = "field", n_transitions: int = 1 << 24,
                         train_steps: int = 96, epochs: int = 96, train_seed: int = 4,
                         gas_weight: float = 1.0, calibrate: bool = True, log=None) -> dict:
    """Train the surrogate on transitions the FP64 integrator generates (ctx):
    a digester field of seed 5 run as the coupling driver runs it (or the
    batched population of seed 2), about n_transitions transitions over
    train_steps coupling steps; particle split 90/5/5 with train_seed; the
    output biases calibrated on half of the validation rows.  Leaves the
    trained weights in sur; returns the training record."""
    import time

    import torch
    dev = "cuda"
    n_train = W.pad_ld((n_transitions + train_steps - 1) // train_steps, 64)
    t0 = time.perf_counter()
    floor = default_floor()
    sur.set_weights(init_params(train_seed), identity_norm(floor))
    if train_data == "field":
        wt = W.digester_field(n_train, seed=5, steps=train_steps)
        states, Ds, ok, T = integrate_field_states(ctx, wt, train_steps)
    else:
        wt = W.batched_population(n_train, seed=2, steps=train_steps)
        states, Ds, ok, T = integrate_states(ctx, wt, train_steps)
    g = np.random.default_rng(train_seed)
    perm = g.permutation(wt.n)
    tr_h = np.sort(perm[: int(0.9 * wt.n)]).astype(np.int32)
    va_h = np.sort(perm[int(0.9 * wt.n): int(0.95 * wt.n)]).astype(np.int32)
    tr, va = torch.from_numpy(tr_h).to(dev), torch.from_numpy(va_h).to(dev)
    out_weight = np.ones(OUT)
    out_weight[[8, 9, 32, 33, 34]] = gas_weight
    norm = fit_norm(sur, states, Ds, T, wt.dt, wt.n, floor, rows=tr, out_weight=out_weight)
    sur.set_weights(init_params(train_seed), norm)
    X, Tg = dataset(sur, states, Ds, T, wt.dt, wt.n, rows=tr)
    # transitions of clean steps only (dataset rows are step-major)
    keep = ok[:, tr_h].reshape(-1)
    kept = torch.from_numpy(np.flatnonzero(keep).astype(np.int32)).to(dev)
    Xk = torch.empty((kept.shape[0], X.shape[1]), dtype=X.dtype, device=dev)
    Tk = torch.empty((kept.shape[0], Tg.shape[1]), dtype=Tg.dtype, device=dev)
    adm1_gather_rows(X, kept, Xk)
    adm1_gather_rows(Tg, kept, Tk)
    X, Tg = Xk, Tk
    Xv, Tv = dataset(sur, states, Ds, T, wt.dt, wt.n, rows=va)
    del states
    gen_s = time.perf_counter() - t0
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist = train(sur, X, Tg, epochs=epochs, batch=8192, lr=1e-3, seed=train_seed, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    steps = epochs * (X.shape[0] // 8192)
    shift = np.zeros(OUT)
    if calibrate:
        half = Xv.shape[0] // 2
        shift = calibrate_output_bias(sur, Xv[:half], Tv[:half])
        Xv, Tv = Xv[half:], Tv[half:]
    val_mse = float(adm1_surrogate_residual_stats(sur.handle, Xv, Tv)[1].mean())
    rec = {"data": train_data, "transitions": int(keep.sum()), "particles": int(wt.n),
           "coupling_steps": train_steps, "epochs": epochs, "steps": steps,
           "seconds": train_s, "data_seconds": gen_s, "loss_first_last": [hist[0], hist[-1]],
           "val_mse": val_mse, "output_bias_shift_max": float(np.abs(shift).max()),
           "train_seed": train_seed, "gas_weight": gas_weight, "calibrated": bool(calibrate)}
    del X, Tg, Xv, Tv
    torch.cuda.empty_cache()
    return rec


def save_checkpoint(path: str, sur: Surrogate, record: dict):
    """Weights (flat FP32 in the ABI's layer order), normalisation and the
    training record, as a NumPy archive without pickled objects."""
    import json
    params, norm = sur.get_weights()
    nd = norm_dict(norm)
    np.savez(path, params=np.asarray(params, np.float32), record=np.array(json.dumps(record)),
             **{k: np.asarray(v) for k, v in nd.items()})


def load_checkpoint(path: str):
    """(params, adm1_mlp_norm, record) of a checkpoint written by
    save_checkpoint."""
    import json
    with np.load(path, allow_pickle=False) as z:
        params = z["params"].astype(np.float32)
        norm = make_norm(z["in_mean"], z["in_sd"], z["out_mean"], z["out_sd"], z["floor"])
        record = json.loads(str(z["record"]))
    if params.size != NPARAMS:
        raise ValueError(f"{path}: {params.size} parameters, expected {NPARAMS}")
    return params, norm, record
