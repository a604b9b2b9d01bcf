"""Benchmark: ADM1 particle-steps per second of the per-particle reaction step.

Workload (default): the batched population of 2^20 particles (per-particle
temperature 30-40 C with Arrhenius-scaled rates, a 5 % feed zone pulsed with
10x substrate on even coupling steps), 10 coupling steps of dt = 1/96 d,
FP64 integrator at rtol 1e-8.  One timed step = one coupling interval of the
whole hot path: the adaptive Rosenbrock step of every particle
(adm1_step_particles) and the tank gas flows (adm1_gas_flux).  Inputs are in
HBM before the timed region.  Warm-up steps run on a copy of the initial
state, which is restored before timing, so the timed steps are the
workload's first K coupling intervals.

Prints one JSON line.  Only one GPU is used; --gpus above 1 exits.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12  # MI355X FP64 vector, FLOP/s
PEAK_HBM = 8.0e12    # bytes/s
# the paper's thread-scaling run (sec. 4.3): CSTR particles of the fixed path
FIXED_PARTICLES = 110_929

# Sources of the step kernel: HBM traffic measured with hardware counters is
# reported only while they are unchanged since the measurement.
STEP_SOURCES = ["adm1_step_sparse2.hip", "adm1_model.h", "adm1_jac_sparse2.inc",
                "adm1_partials.inc", "adm1_stoich.inc", "adm1_devparams.h", "adm1_rodas4.h",
                "adm1_kernels.h"]
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_step_sparse2_batched_2e20.md")
# the same for the fixed-step kernels (whose source file holds the other
# one-lane kernels too: any change there drops the measured figure)
FIXED_SOURCES = ["adm1_kernels.hip", "adm1_fixed.h", "adm1_model.h", "adm1_partials.inc",
                 "adm1_stoich.inc", "adm1_devparams.h", "adm1_kernels.h", "adm1_count.h",
                 "adm1_rodas4.h"]
FIXED_PROFILE = os.path.join(ROOT, "profiles", "k_fixed_cstr_110929.md")


def step_source_hash(sources=None) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in STEP_SOURCES if sources is None else sources:
        with open(os.path.join(ROOT, "paper_2311_08927_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(K: int, launch: str):
    """Calibrated HBM bytes per launch of the step kernel, averaged over the
    first K coupling intervals, from the committed counter summary (one value
    per interval of the profiled run); None when the kernel sources changed
    since the counters were taken or the profile covers fewer intervals."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    kv = dict(re.findall(r"^- (\w+): `([^`]*)`", text, flags=re.M))
    if kv.get("kernel_source_sha256") != step_source_hash() or kv.get("launch") != launch:
        return None
    try:
        per = [float(v) for v in kv["traffic_bytes_per_interval"].split(",")]
    except (KeyError, ValueError):
        return None
    if K > len(per):
        return None
    return sum(per[:K]) / K


def fixed_traffic(shape: str):
    """Calibrated HBM bytes per launch of the fixed-step kernel for `shape`
    (method|particles|substeps|interval), from the committed counter summary;
    None when its sources changed since the counters were taken or the
    summary covers another shape."""
    try:
        text = open(FIXED_PROFILE).read()
    except OSError:
        return None
    kv = dict(re.findall(r"^- (\w+): `([^`]*)`", text, flags=re.M))
    if kv.get("kernel_source_sha256") != step_source_hash(FIXED_SOURCES) or \
            kv.get("shape") != shape:
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_probe(mib: int, dev) -> None:
    """One device-to-device copy of `mib` MiB: the known-size kernel whose
    byte counters calibrate those of the kernels around it."""
    import torch
    if mib <= 0:
        return
    src = torch.ones(mib << 18, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed coupling steps (default 10 for the FP64 path, 96 for the "
                         "surrogate)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=None,
                    help="particles (default 2^20 for the FP64 path, 2^24 for the surrogate)")
    ap.add_argument("--path", choices=["fp64", "surrogate", "fixed"], default="fp64",
                    help="fp64: adaptive Rodas4 step (default); surrogate: gated MLP against "
                         "it; fixed: the paper's fixed-step explicit scheme")
    ap.add_argument("--method", choices=["euler", "rk4"], default="euler",
                    help="fixed path: explicit update")
    ap.add_argument("--interval-s", type=float, default=0.5,
                    help="fixed path: coupling interval in seconds (the paper's Dt)")
    ap.add_argument("--substeps", type=int, default=10,
                    help="fixed path: explicit steps per interval (the paper's ten)")
    ap.add_argument("--train-epochs", type=int, default=96)
    ap.add_argument("--gate-ion", type=float, default=1e-2,
                    help="surrogate gate: tolerance of the proposed ions and S_h2")
    ap.add_argument("--gate-closure", type=float, default=5e-4,
                    help="surrogate gate: tolerance of the COD / nitrogen closure")
    ap.add_argument("--fallback-rtol", type=float, default=1e-4,
                    help="surrogate: tolerance of the exact integration of rejected particles")
    ap.add_argument("--fair-rtols", type=str, default="1e-2,1e-3,1e-4,1e-5,1e-6",
                    help="surrogate: looser FP64 tolerances timed on the same field; the "
                         "loosest one within 1e-3 of the rtol-1e-8 run in tank methane flow "
                         "and pH (p99) is the fair baseline ('' to skip)")
    ap.add_argument("--train-data", choices=["field", "batched"], default="field",
                    help="surrogate: transitions to train on (field: a digester field of "
                         "another seed, run as the coupling driver runs it; batched: the "
                         "batched population)")
    ap.add_argument("--gas-weight", type=float, default=1.0,
                    help="surrogate: training-loss weight of the outputs that set the "
                         "methane flow (S_ch4, S_IC and the three gas-phase states)")
    ap.add_argument("--train-steps", type=int, default=96,
                    help="surrogate: coupling steps of the training runs (the particle "
                         "count is chosen for about 2^24 transitions)")
    ap.add_argument("--train-seed", type=int, default=4,
                    help="surrogate: seed of the initial weights and of the data split")
    ap.add_argument("--calibrate", type=int, default=1, choices=[0, 1],
                    help="surrogate: shift the output biases by the mean validation residual")
    ap.add_argument("--burn-in", type=int, default=2,
                    help="surrogate path: untimed FP64 steps before the comparison")
    ap.add_argument("--checkpoint", default=None,
                    help="surrogate path: load the network from this checkpoint instead of "
                         "training it (paper_2311_08927_amd/train_surrogate.py writes one)")
    ap.add_argument("--gate-sweep", default="3e-3:3e-4,1e-3:1e-4,3e-4:3e-5,1e-4:1e-5",
                    help="surrogate path: further gate settings tol_ion:tol_closure, "
                         "comma separated, timed on the same field (the trade-off curve)")
    ap.add_argument("--headline", type=int, default=1, choices=[0, 1],
                    help="fp64 path: also run the gated-surrogate comparison on the 2^24 "
                         "digester field over 96 coupling steps from the committed "
                         "checkpoint and report it under 'headline'")
    ap.add_argument("--headline-n", type=int, default=1 << 24)
    ap.add_argument("--headline-resync", default="",
                    help="headline: periods R (comma separated) of surrogate runs whose "
                         "every R-th step is the exact FP64 step of all particles")
    ap.add_argument("--headline-steps", type=int, default=96)
    ap.add_argument("--variant", type=int, default=-1)
    ap.add_argument("--rate-precision", type=int, default=0, choices=[0, 1],
                    help="1: rates and eq. 2 assembly in FP32 (the FP32-rate experiment)")
    ap.add_argument("--blocks-per-cu", type=int, default=0,
                    help="resident waves per CU of the persistent step kernel (0: library "
                         "default)")
    ap.add_argument("--order", choices=["cost", "index"], default="cost",
                    help="work-queue order of the step kernel (cost: expected step count "
                         "from the previous interval, largest first)")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--autotune", type=int, default=1, choices=[0, 1],
                    help="fp64 path: pick the step kernel's launch configuration with the "
                         "autotuner on a sample of the workload before timing (cached)")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="particles of the oracle CPU-baseline sample (0: skip; default "
                         "163,840 particle-steps over the timed horizon)")
    ap.add_argument("--cpu-steps", type=int, default=None,
                    help="coupling steps of the CPU sample (default: the timed steps)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the timed region, one device-to-device copy of this size "
                         "(the known-size kernel that calibrates HBM byte counters)")
    return ap.parse_args()


def autotune_sample(ctx, w, rtol):
    """Pick the step kernel's launch configuration (paper_2311_08927_amd
    .autotune) on a seeded sample of the workload that keeps its feed-zone
    share: 65,536 particles (one wave per SIMD for the one-lane layouts), a
    cold coupling interval and two warm ones per candidate (the timed run is
    mostly warm intervals, where the service phase weighs more)."""
    import torch

    from paper_2311_08927_amd import autotune as AT
    from paper_2311_08927_amd import workloads as W
    rng = np.random.default_rng(77)
    m = min(65536, w.n)
    idx = np.sort(rng.choice(w.n, m, replace=False))
    sub = W.subset(w, idx)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")  # noqa: E731
    res = AT.autotune(ctx, t(sub.X), t(sub.T), t(sub.D_at(0)), t(sub.fidx), t(sub.feed),
                      sub.dt, n=sub.n, tag=f"batched-sample-{m}-x3", intervals=3)
    res["sample"] = (f"{m} seeded particles of the workload, a cold coupling interval and "
                     f"two warm ones per candidate, median of 2")
    return res


def cpu_baseline(w, rtol, n_sample, steps):
    """The oracle, as it stands, on a stratified sample of the same workload."""
    from oracle.adm1 import Oracle
    from paper_2311_08927_amd import workloads as W
    rng = np.random.default_rng(123)
    zone = np.flatnonzero(w.zone)
    other = np.flatnonzero(~w.zone)
    nz = max(1, int(round(n_sample * len(zone) / w.n)))
    idx = np.sort(np.concatenate([rng.choice(zone, nz, replace=False),
                                  rng.choice(other, n_sample - nz, replace=False)]))
    sub = W.subset(w, idx)
    orc = Oracle(W.params_path(), rtol=rtol, atol=W.atol_vector(rtol))
    cores = len(os.sched_getaffinity(0))
    X = sub.X.copy()
    H = np.full(sub.ld, -1.0)
    hl = np.full(sub.ld, -1.0)
    t0 = time.perf_counter()
    for s in range(steps):
        orc.step(X, sub.T, sub.D_at(s), sub.fidx, sub.feed, sub.dt, H=H, hlast=hl, n=sub.n,
                 nthreads=cores)
    el = time.perf_counter() - t0
    rec = {"value": sub.n * steps / el, "unit": "particle-steps/s", "cores": cores,
           "kind": "oracle",
           "sample": f"{sub.n} particles ({nz} in the feed zone) x {steps} coupling steps "
                     f"of the same workload, std::thread-style equal chunks, {el:.1f} s"}
    # the same oracle on one thread, every 32nd particle of the sample
    one = W.subset(w, idx[::32])
    X1 = one.X.copy()
    H1, hl1 = np.full(one.ld, -1.0), np.full(one.ld, -1.0)
    t1 = time.perf_counter()
    for s in range(steps):
        orc.step(X1, one.T, one.D_at(s), one.fidx, one.feed, one.dt, H=H1, hlast=hl1,
                 n=one.n, nthreads=1)
    el1 = time.perf_counter() - t1
    single = {"value": one.n * steps / el1, "unit": "particle-steps/s", "cores": 1,
              "sample": f"every 32nd particle of that sample ({one.n}) x {steps} coupling "
                        f"steps, {el1:.1f} s"}
    return rec, idx, X[:, :sub.n], single


def main():
    args = parse()
    if args.n is None:
        args.n = {"surrogate": 1 << 24, "fixed": FIXED_PARTICLES}.get(args.path, 1 << 20)
    if args.steps is None:
        args.steps = {"surrogate": 96, "fixed": 100}.get(args.path, 10)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the "
              "particle step shards by index range with no exchange besides four gas "
              "totals, so N GPUs would each run this single-GPU path on n/N particles.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2311_08927_amd import adm1 as A
    from paper_2311_08927_amd import flops as F
    from paper_2311_08927_amd import workloads as W
    if args.path == "surrogate":
        return surrogate_main(args)
    if args.path == "fixed":
        return fixed_main(args)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = W.batched_population(args.n, seed=2, steps=args.steps)
    ctx = A.Context(w.ld, rtol=args.rtol, atol=W.atol_vector(args.rtol), variant=args.variant,
                    rate_precision=args.rate_precision)
    A.adm1_set_order(ctx.handle, A.ORDER_COST if args.order == "cost" else A.ORDER_INDEX)
    tune = None
    if args.blocks_per_cu > 0:
        A.adm1_set_launch(ctx.handle, A.VARIANT_SPARSE2, args.blocks_per_cu)
    elif args.variant < 0 and args.autotune:
        tune = autotune_sample(ctx, w, args.rtol)
    launch = ("tuned " + ":".join(map(str, tune["choice"]))) if tune else \
        f"variant {args.variant}, blocks per CU {args.blocks_per_cu}"
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    X0 = t(w.X)
    X = X0.clone()
    T = t(w.T)
    D_even, D_odd = t(w.D_at(0)), t(w.D_at(1))
    fidx, S_in = t(w.fidx), t(w.feed)
    H = torch.full((w.n,), -1.0, dtype=torch.float64, device=dev)
    hl = torch.full((w.n,), -1.0, dtype=torch.float64, device=dev)
    status = torch.zeros(w.n, dtype=torch.uint8, device=dev)
    K = args.steps
    nsteps = torch.zeros((K, 3, w.ld), dtype=torch.int32, device=dev)
    V_liq = torch.full((w.n,), 3400.0, dtype=torch.float64, device=dev)
    q_gas = torch.empty(w.n, dtype=torch.float64, device=dev)
    q_ch4 = torch.empty(w.n, dtype=torch.float64, device=dev)
    totals = torch.empty((K, 4), dtype=torch.float64, device=dev)
    feeds = [A.feed_struct(D_even, fidx, S_in), A.feed_struct(D_odd, fidx, S_in)]
    aux = A.adm1_aux(H.data_ptr(), hl.data_ptr())
    stream = torch.cuda.current_stream()

    def one_step(k, ns, tot):
        A.adm1_step_particles(ctx.handle, X, w.ld, T, feeds[k % 2], w.dt, w.n, aux, status, ns,
                              stream)

    def gas(k, tot):
        A.adm1_gas_flux(ctx.handle, X, w.ld, T, V_liq, w.n, q_gas, q_ch4, tot, stream)

    # warm-up on a copy, then restore the initial state and warm starts
    for k in range(args.warmup):
        one_step(k, nsteps[0], totals[0])
        gas(k, totals[0])
    torch.cuda.synchronize()
    X.copy_(X0)
    H.fill_(-1.0)
    hl.fill_(-1.0)
    nsteps.zero_()
    copy_probe(args.copy_probe_mib, dev)
    torch.cuda.synchronize()

    ev_s = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    ev_e = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for k in range(K):
        ev_s[k].record(stream)
        one_step(k, nsteps[k], totals[k])
        ev_e[k].record(stream)
        gas(k, totals[k])
        print(f"# step {k} enqueued", file=sys.stderr, flush=True)
    end.record(stream)
    end.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(end)
    step_ms = [ev_s[k].elapsed_time(ev_e[k]) for k in range(K)]

    st = status.cpu().numpy()
    ns = nsteps.cpu().numpy().astype(np.int64)
    acc = int(ns[:, 0, :w.n].sum())
    rej = int(ns[:, 1, :w.n].sum())
    newt = int(ns[:, 2, :w.n].sum())
    flop = F.total_flops(acc + rej, newt, w.n * K)
    kern_s = sum(step_ms) / 1e3
    achieved = flop / kern_s
    value = w.n * K / (total_ms / 1e3)
    traffic = None
    if args.n == 1 << 20 and args.rtol == 1e-8 and args.rate_precision == 0 and \
            args.order == "cost":
        traffic = measured_traffic(K, launch)
    size = "2^20" if w.n == 1 << 20 else str(w.n)
    out = {
        "metric": "ADM1 particle-steps/sec (FP64 integrator vs gated surrogate) at stated error",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": total_ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.rate_precision == 0 else "f64 (rates f32)",
        "data": "synthetic",
        "config": {"workload": f"batched ADM1 population: {size} particles, T U(30,40) C, "
                               f"5% pulsed feed zone, {K} coupling steps of 1/96 d from a "
                               f"cold start, rtol {args.rtol:g}",
                   "particles": w.n, "coupling_steps": K, "dt_days": w.dt, "rtol": args.rtol,
                   "path": "fp64 integrator" if args.rate_precision == 0 else
                   "fp64 integrator, fp32 rates", "variant": args.variant,
                   "queue_order": args.order,
                   "launch": tune["layout"] if tune else launch,
                   "autotune": None if tune is None else
                   {"sample": tune["sample"], "cached": bool(tune.get("cached")),
                    "source": tune.get("source", "tuned in this run"),
                    "timings_ms": tune["timings_ms"]}},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": traffic,
                     "kernel": "adm1 step (k_step*)",
                     "avg_launch_ms": sum(step_ms) / K,
                     "flops_per_launch": flop / K},
        "detail": {"accepted_steps": acc, "rejected_steps": rej, "newton_iters": newt,
                   "attempts_per_particle_step": (acc + rej) / (w.n * K),
                   "status_counts": np.bincount(st & 0x7F, minlength=5).tolist(),
                   "hbm_bytes_per_particle_step": F.BYTES_PER_PARTICLE_STEP,
                   "hbm_frac": w.n * F.BYTES_PER_PARTICLE_STEP / (sum(step_ms) / K / 1e3)
                   / PEAK_HBM,
                   "step_ms": step_ms, "step_ms_median": float(np.median(step_ms)),
                   "wall_s": wall,
                   "cold_interval_ms": step_ms[0],
                   "warm_interval_mean_ms": (sum(step_ms[1:]) / (K - 1)) if K > 1 else None},
    }
    cpu_steps = args.cpu_steps or K
    n_sample = args.cpu_sample
    if n_sample is None:
        n_sample = int(min(16384, max(1024, round(163840 / cpu_steps))))
    if n_sample > 0:
        out["cpu_baseline"], idx, Xo, single = cpu_baseline(w, args.rtol, n_sample, cpu_steps)
        out["detail"]["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
        out["detail"]["cpu_single_thread"] = single
        if cpu_steps == K:
            # the timed run's own final states against the oracle's on the
            # sample (the parity metric of the tests)
            xg = X[:, torch.from_numpy(idx).to(dev)].cpu().numpy()
            nom = W.nominal()["state"][:, None]
            rel = np.abs(xg - Xo) / np.maximum(np.abs(Xo), 1e-4 * nom)
            out["detail"]["parity_vs_oracle_sample"] = {
                "max_rel": float(rel.max()), "particles": int(len(idx)), "bar": 1e-6,
                "metric": "|x_gpu - x_oracle| / max(|x_oracle|, 1e-4 x_nom) after the timed "
                          "coupling steps"}
        out["detail"]["gpu_over_cpu_horizon"] = (f"both over coupling steps 0..{K - 1}"
                                                 if cpu_steps == K else
                                                 f"GPU {K} steps, CPU {cpu_steps} steps")
    if args.headline:
        del X, X0, H, hl, status, nsteps, q_gas, q_ch4, totals, V_liq, T, fidx, S_in
        ctx.close()
        torch.cuda.empty_cache()
        out["headline"] = headline(args)
    print(json.dumps(out))


def headline(args):
    """The metric's comparison at the size it names: the 2^24-particle
    digester field over 96 coupling steps (one simulated day), the FP64
    integrator (rtol 1e-8) against the gated surrogate loaded from the
    committed checkpoint, its gate trade-off and the fair FP64 baseline."""
    from paper_2311_08927_amd import adm1 as A
    from paper_2311_08927_amd import surrogate as S
    from paper_2311_08927_amd import workloads as W
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    if not os.path.exists(CHECKPOINT):
        return {"skipped": f"no checkpoint at {os.path.relpath(CHECKPOINT, ROOT)}"}
    t0 = time.perf_counter()
    ld = W.pad_ld(args.headline_n)
    ctx = A.Context(ld, rtol=1e-8, atol=W.atol_vector(1e-8), variant=args.variant)
    ctx_fb = A.Context(ld, rtol=args.fallback_rtol, atol=W.atol_vector(args.fallback_rtol),
                       variant=args.variant)
    sur = S.Surrogate(ctx_fb, ld, 8192)
    params, norm, rec = S.load_checkpoint(CHECKPOINT)
    sur.set_weights(params, norm)
    gates = [(args.gate_ion, args.gate_closure)] + [
        tuple(float(v) for v in g.split(":")) for g in args.gate_sweep.split(",") if g.strip()]
    resyncs = [int(v) for v in args.headline_resync.split(",") if v.strip()]
    res = field_comparison(args, args.headline_n, args.headline_steps, sur, ctx, log, gates,
                           [1e-2, 1e-3, 1e-4, 1e-6], resyncs=resyncs)
    sur.close()
    ctx_fb.close()
    ctx.close()
    res["checkpoint"] = {"file": os.path.relpath(CHECKPOINT, ROOT),
                         "written_by": rec.get("command"), "val_mse": rec.get("val_mse"),
                         "transitions": rec.get("transitions"), "epochs": rec.get("epochs")}
    res["wall_seconds"] = time.perf_counter() - t0
    return res


def fixed_cpu_baseline(w, dt, substeps, method, n_sample, steps):
    """The oracle's fixed-step integrator, as it stands, on a seeded sample of
    the same population: equal particle chunks over all host cores (the
    paper's CPU parallelisation, sec. 4.3), through the oracle's own threaded
    C loop."""
    from oracle.adm1 import Oracle
    from paper_2311_08927_amd import workloads as W
    orc = Oracle(W.params_path(), rtol=1e-8, atol=W.atol_vector(1e-8))
    idx = np.sort(np.random.default_rng(123).choice(w.n, min(n_sample, w.n), replace=False))
    sub = W.subset(w, idx)
    cores = len(os.sched_getaffinity(0))
    X = sub.X.copy()
    t0 = time.perf_counter()
    for _ in range(steps):
        orc.run_fixed(X, sub.T, sub.D, sub.fidx, sub.feed, dt, substeps, method, n=sub.n,
                      nthreads=cores)
    el = time.perf_counter() - t0
    return {"value": sub.n * steps / el, "unit": "particle-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{sub.n} particles x {steps} coupling intervals of the same "
                      f"population, equal particle chunks over {cores} threads, {el:.1f} s"}


def fixed_main(args):
    """The paper's own fixed-step scheme (sec. 2.3: synchronised coupling steps
    small enough that no step control is needed; sec. 4.3: 110,929 particles
    of the CSTR case, Dt = 0.5 s in ten internal steps).  A step of the metric
    is one coupling interval of one particle; HIP events bracket every launch
    on the launching stream."""
    import torch

    from paper_2311_08927_amd import adm1 as A
    from paper_2311_08927_amd import flops as F
    from paper_2311_08927_amd import workloads as W
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = W.cstr_population(args.n, seed=1)
    dt = args.interval_s / 86400.0
    meth = A.FIXED_EULER if args.method == "euler" else A.FIXED_RK4
    ctx = A.Context(w.ld, rtol=1e-8, atol=W.atol_vector(1e-8),
                    rate_precision=args.rate_precision)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    X0 = t(w.X)
    X = X0.clone()
    T, D, fidx, S_in = t(w.T), t(w.D), t(w.fidx), t(w.feed)
    H = torch.full((w.n,), -1.0, dtype=torch.float64, device=dev)
    status = torch.zeros(w.n, dtype=torch.uint8, device=dev)
    K = args.steps
    newton = torch.zeros((K, w.n), dtype=torch.int32, device=dev)
    feed = A.feed_struct(D, fidx, S_in)
    stream = torch.cuda.current_stream()

    def one(k):
        A.adm1_step_fixed(ctx.handle, X, w.ld, T, feed, dt, args.substeps, meth, w.n, H,
                          status, newton[k], stream)

    for k in range(args.warmup):
        one(0)
    torch.cuda.synchronize()
    X.copy_(X0)
    H.fill_(-1.0)
    copy_probe(args.copy_probe_mib, dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(K)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for k in range(K):
        ev[k][0].record(stream)
        one(k)
        ev[k][1].record(stream)
    end.record(stream)
    end.synchronize()
    print(f"# {K} intervals done", file=sys.stderr, flush=True)
    total_ms = start.elapsed_time(end)
    launch_ms = [a.elapsed_time(b) for a, b in ev]
    newt = int(newton.sum().item())
    flop = F.fixed_flops(args.method, args.substeps, newt, w.n * K)
    achieved = flop / (sum(launch_ms) / 1e3)
    value = w.n * K / (total_ms / 1e3)
    st = status.cpu().numpy()
    traffic = None
    if args.rate_precision == 0:
        traffic = fixed_traffic(f"{args.method}|{w.n}|{args.substeps}|{args.interval_s:g}")
    out = {
        "metric": "ADM1 particle-steps/sec (FP64 integrator vs gated surrogate) at stated error",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": total_ms / K,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.rate_precision == 0 else "f64 (rates f32)",
        "data": "synthetic",
        "config": {"workload": f"CSTR population of the paper's parallel benchmark shape: "
                               f"{w.n} particles, coupling interval {args.interval_s:g} s "
                               f"in {args.substeps} explicit {args.method} steps, "
                               f"{K} intervals",
                   "path": "fixed-step explicit scheme", "method": args.method,
                   "substeps": args.substeps, "interval_s": args.interval_s},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": traffic,
                     "kernel": f"k_fixed ({args.method})",
                     "avg_launch_ms": sum(launch_ms) / K, "flops_per_launch": flop / K},
        "detail": {"substeps_per_s": value * args.substeps,
                   "newton_per_particle_interval": newt / (w.n * K),
                   "status_counts": np.bincount(st & 0x7F, minlength=5).tolist(),
                   "hbm_bytes_per_particle_step": F.BYTES_FIXED,
                   "hbm_frac": w.n * F.BYTES_FIXED / (sum(launch_ms) / K / 1e3) / PEAK_HBM},
    }
    n_sample = 65536 if args.cpu_sample is None else args.cpu_sample
    if n_sample > 0:
        out["cpu_baseline"] = fixed_cpu_baseline(w, dt, args.substeps, args.method,
                                                 n_sample, args.cpu_steps or 10)
        out["detail"]["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    print(json.dumps(out))


CHECKPOINT = os.path.join(ROOT, "paper_2311_08927_amd", "data", "surrogate_field.npz")


def field_comparison(args, n, steps, sur, ctx, log, gates=None, fair_rtols=None,
                     fp64_nsteps=True, resyncs=()):
    """Gated surrogate against the FP64 path on the digester field (the
    coupling loop: feed mask, step, gas flux; advection between steps), from
    the same burned-in states.  Positions of every step are advected once
    up front (the flow does not depend on the states), so every path sees
    the same particles in the inlet.  Each path's step + gas flux is replayed
    from a captured HIP graph; the feed mask before it is timed with it.
    gates: list of (tol_ion, tol_closure) settings of the surrogate (the
    first is the reported one); fair_rtols: looser FP64 tolerances, the
    loosest within 1e-3 of the rtol-1e-8 run in tank methane flow (every step)
    and pH (p99) being the fair baseline.  resyncs: periods R of a surrogate
    path (first gate) whose every R-th step is the exact FP64 step of all
    particles instead."""
    import torch

    from paper_2311_08927_amd import adm1 as A
    from paper_2311_08927_amd import flops as F
    from paper_2311_08927_amd import surrogate as S
    from paper_2311_08927_amd import workloads as W
    dev = torch.device("cuda:0")
    gates = gates or [(args.gate_ion, args.gate_closure)]
    fair_rtols = [] if fair_rtols is None else fair_rtols
    wd = W.digester_field(n, seed=3, steps=args.burn_in + steps)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    X = t(wd.X)
    T = t(wd.T)
    S_in = t(wd.feed)
    pos = t(wd.extra["pos"])
    del wd.X
    flow = A.make_flow(wd.extra["flow"])
    D = torch.zeros(wd.n, dtype=torch.float64, device=dev)
    fidx = torch.zeros(wd.n, dtype=torch.int32, device=dev)
    V = torch.full((wd.n,), wd.extra["V_p"], dtype=torch.float64, device=dev)
    H = torch.full((wd.n,), -1.0, dtype=torch.float64, device=dev)
    hl = torch.full((wd.n,), -1.0, dtype=torch.float64, device=dev)
    status = torch.zeros(wd.n, dtype=torch.uint8, device=dev)
    dt_s = wd.dt * 86400.0
    sub = W.advect_substeps(dt_s)

    def mask(p):
        A.adm1_feed_mask(p, wd.ld, wd.n, W.INLET_Z, W.INLET_R, 1.0, 1, 0, D, fidx)

    # burn-in with the FP64 path (untimed)
    for k in range(args.burn_in):
        mask(pos)
        ctx.step(X, T, D, fidx, S_in, wd.dt, n=wd.n, H=H, hlast=hl, status=status)
        A.adm1_advect(pos, wd.ld, wd.n, flow, dt_s, sub)
    # positions at the start of every compared step (advected once)
    t_adv = time.perf_counter()
    pos_k = []
    for k in range(steps):
        pos_k.append(pos.clone())
        A.adm1_advect(pos, wd.ld, wd.n, flow, dt_s, sub)
    torch.cuda.synchronize()
    adv_s = time.perf_counter() - t_adv
    log(f"# field {wd.n}: burn-in and {steps} advections done ({adv_s:.1f} s)")
    X0, H0, hl0 = X.clone(), H.clone(), hl.clone()
    tot_g = torch.zeros(4, dtype=torch.float64, device=dev)
    fb_g = torch.zeros(1, dtype=torch.int32, device=dev)
    route_g = torch.zeros(wd.n, dtype=torch.uint8, device=dev)
    ns_g = torch.zeros((3, wd.ld), dtype=torch.int32, device=dev) if fp64_nsteps else None
    feed = A.feed_struct(D, fidx, S_in)
    aux = A.adm1_aux(H.data_ptr(), hl.data_ptr())
    cap = torch.cuda.Stream()
    graphs, ctxs = {}, {}
    graphs["fp64"] = A.adm1_graph_capture_step(ctx.handle, X, wd.ld, T, feed, wd.dt, wd.n, aux,
                                               status, ns_g, V, None, None, tot_g, cap)
    for gi, (ti, tc) in enumerate(gates):
        graphs[f"sur{gi}"] = S.adm1_surrogate_graph_capture_step(
            sur.handle, X, wd.ld, T, feed, wd.dt, wd.n, S.adm1_gate(5.0, ti, tc), aux, status,
            None, route_g, fb_g, V, None, None, tot_g, cap)
    for r in fair_rtols:
        c = A.Context(wd.ld, rtol=r, atol=W.atol_vector(r), variant=args.variant)
        ctxs[r] = c
        graphs[f"fp64@{r:g}"] = A.adm1_graph_capture_step(c.handle, X, wd.ld, T, feed, wd.dt,
                                                          wd.n, aux, status, None, V, None,
                                                          None, tot_g, cap)
    paths = list(graphs) + [f"sur0+exact/{R}" for R in resyncs]
    K = steps

    def graph_of(path, k):
        if path.startswith("sur0+exact/"):
            R = int(path.split("/")[1])
            return graphs["fp64"] if (k + 1) % R == 0 else graphs["sur0"]
        return graphs[path]
    tot = {p: torch.zeros((K, 4), dtype=torch.float64, device=dev) for p in paths}
    fb = {p: torch.zeros(K, dtype=torch.int32, device=dev) for p in paths}
    ms, launch_ms, out_H, out_X = {}, {}, {}, {}
    attempts = torch.zeros(3, dtype=torch.int64, device=dev)
    # audit: 4,096 seeded particles per surrogate step integrated exactly
    # from their pre-step states (outside the timed region)
    aud = torch.from_numpy(np.sort(np.random.default_rng(7).choice(wd.n, 4096, replace=False)))
    aud = aud.to(dev)
    nom = torch.from_numpy(W.nominal()["state"]).to(dev)[:, None]
    audit = {}
    stream = torch.cuda.current_stream()
    for path in paths:
        # one untimed warm-up replay of the path's first step, then the
        # burned-in state again
        X.copy_(X0); H.copy_(H0); hl.copy_(hl0)
        mask(pos_k[0])
        A.adm1_graph_launch(graph_of(path, 0), stream)
        torch.cuda.synchronize()
        X.copy_(X0); H.copy_(H0); hl.copy_(hl0)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(K)]
        amax, ap99 = [], []
        for k in range(K):
            ev[k][0].record()
            mask(pos_k[k])
            if path == "sur0":
                pre = (X.index_select(1, aud), H.index_select(0, aud), hl.index_select(0, aud),
                       D.index_select(0, aud), fidx.index_select(0, aud))
            A.adm1_graph_launch(graph_of(path, k), stream)
            ev[k][1].record()
            if path == "fp64" and ns_g is not None:
                attempts += ns_g[:, :wd.n].sum(dim=1)
            if path == "sur0":
                Xa, Ha, hla, Da, fia = pre
                ctx.step(Xa, T.index_select(0, aud), Da, fia, S_in, wd.dt, n=aud.numel(),
                         H=Ha, hlast=hla)
                acc = route_g.index_select(0, aud).bool()
                err = ((X.index_select(1, aud) - Xa).abs() /
                       torch.maximum(Xa.abs(), 1e-4 * nom)).amax(dim=0)[acc]
                amax.append(float(err.max()) if err.numel() else 0.0)
                ap99.append(float(torch.quantile(err.float(), 0.99)) if err.numel() else 0.0)
            tot[path][k].copy_(tot_g)
            if graph_of(path, k) is graphs["fp64"] and path != "fp64":
                fb[path][k] = wd.n          # every particle integrated exactly
            else:
                fb[path][k:k + 1].copy_(fb_g)
        torch.cuda.synchronize()
        launch_ms[path] = [e0.elapsed_time(e1) for e0, e1 in ev]
        ms[path] = sum(launch_ms[path])
        out_H[path] = H.clone()
        if path in ("fp64", "sur0"):
            out_X[path] = X.clone()
        if path == "sur0":
            audit = {"sample": "4096 seeded particles per step; accepted ones integrated "
                               "exactly from their pre-step states",
                     "rel_err_max": amax, "rel_err_p99": ap99}
        log(f"# {path}: {K} steps, {ms[path]:.0f} ms")
    for gph in graphs.values():
        A.adm1_graph_destroy(gph)
    for c in ctxs.values():
        c.close()
    ch4_ref = tot["fp64"][:, 2].cpu().numpy()
    ph_ref = -torch.log10(out_H["fp64"])
    stride = max(1, wd.n >> 22)

    def errors(path):
        c = tot[path][:, 2].cpu().numpy()
        e_ch4 = np.abs(c - ch4_ref) / np.abs(ch4_ref)
        e_ph = ((-torch.log10(out_H[path]) - ph_ref).abs() / ph_ref).float()
        return e_ch4, float(torch.quantile(e_ph[::stride], 0.99)), float(e_ph.max())

    rate = lambda p: wd.n * K / (ms[p] / 1e3)  # noqa: E731

    def step_ms(p):
        """Mean and median over the K timed replays of a path (ms)."""
        v = np.asarray(launch_ms[p])
        return {"mean": float(v.mean()), "median": float(np.median(v)), "n": int(v.size)}
    v64 = rate("fp64")
    sweep, fair = [], None
    for r in sorted(fair_rtols, reverse=True):
        e_ch4, p99, pmax = errors(f"fp64@{r:g}")
        row = {"rtol": r, "particle_steps_per_s": rate(f"fp64@{r:g}"),
               "step_ms": step_ms(f"fp64@{r:g}"),
               "tank_methane_rel_err_max": float(e_ch4.max()), "ph_rel_err_p99": p99,
               "ph_rel_err_max": pmax}
        sweep.append(row)
        if fair is None and row["tank_methane_rel_err_max"] <= 1e-3 and p99 <= 1e-3:
            fair = row
    gate_rows = []
    for gi, (ti, tc) in enumerate(gates):
        e_ch4, p99, pmax = errors(f"sur{gi}")
        v = rate(f"sur{gi}")
        fbf = (fb[f"sur{gi}"].cpu().numpy() / wd.n)
        gate_rows.append({"tol_ion": ti, "tol_closure": tc, "particle_steps_per_s": v,
                          "step_ms": step_ms(f"sur{gi}"), "speedup_vs_fp64": v / v64,
                          "speedup_vs_fair": None if fair is None else
                          v / fair["particle_steps_per_s"],
                          "fallback_fraction_mean": float(fbf.mean()),
                          "tank_methane_rel_err_max": float(e_ch4.max()),
                          "tank_methane_steps_within_1e-3": int((e_ch4 <= 1e-3).sum()),
                          "ph_rel_err_p99": p99, "ph_rel_err_max": pmax,
                          "meets_1e-3": bool(e_ch4.max() <= 1e-3 and p99 <= 1e-3)})
    resync_rows = []
    for R in resyncs:
        path = f"sur0+exact/{R}"
        e_ch4, p99, pmax = errors(path)
        v = rate(path)
        resync_rows.append({"period": R, "tol_ion": gates[0][0], "tol_closure": gates[0][1],
                            "particle_steps_per_s": v, "step_ms": step_ms(path),
                            "speedup_vs_fp64": v / v64,
                            "speedup_vs_fair": None if fair is None else
                            v / fair["particle_steps_per_s"],
                            "tank_methane_rel_err_max": float(e_ch4.max()),
                            "tank_methane_steps_within_1e-3": int((e_ch4 <= 1e-3).sum()),
                            "ph_rel_err_p99": p99, "ph_rel_err_max": pmax,
                            "meets_1e-3": bool(e_ch4.max() <= 1e-3 and p99 <= 1e-3)})
    e_ch4, p99, pmax = errors("sur0")
    # per-state error of the surrogate's final states (every 64th particle)
    sl = slice(0, wd.n, 64)
    rel = ((out_X["sur0"][:, sl] - out_X["fp64"][:, sl]).abs() /
           torch.maximum(out_X["fp64"][:, sl].abs(), 1e-4 * nom)).float()
    # FP64 path roofline: the flop model on its own attempt counts
    acc, rej, newt = [int(v) for v in attempts.cpu().tolist()]
    fp64_flop = F.total_flops(acc + rej, newt, wd.n * K) if fp64_nsteps else None
    # forward kernel alone (MFMA roofline)
    Xf = sur.featurize(X0, T, D, wd.dt, wd.n)
    sur.forward(Xf)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sur.forward(Xf)
    e1.record()
    e1.synchronize()
    fwd_ms = e0.elapsed_time(e1)
    mlp_flop = 2.0 * (38 * 256 + 3 * 256 * 256 + 256 * 35) * wd.n
    res = {
        "workload": f"digester field: {wd.n} particles in the r 0.1 m, h 0.3 m cylinder, "
                    f"seeded flow, top-inlet pulse feed, 308.5 K, {K} coupling steps of "
                    f"1/96 d after {args.burn_in} FP64 burn-in steps; each path's step "
                    f"captured in a HIP graph",
        "particles": wd.n, "coupling_steps": K,
        "fp64": {"rtol": 1e-8, "particle_steps_per_s": v64, "ms_per_step": ms["fp64"] / K,
                 "step_ms": step_ms("fp64"),
                 "roofline": None if fp64_flop is None else
                 {"bound": "alu", "achieved": fp64_flop / (ms["fp64"] / 1e3) / 1e12,
                  "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                  "frac": fp64_flop / (ms["fp64"] / 1e3) / PEAK_FP64,
                  "kernel": "k_step_sparse2 (with the feed mask and gas flux in the timed "
                            "region)",
                  "attempts_per_particle_step": (acc + rej) / (wd.n * K)}},
        "surrogate": dict(gate_rows[0], **{
            "ms_per_step": ms["sur0"] / K, "fallback_rtol": args.fallback_rtol,
            "fallback_fraction": (fb["sur0"].cpu().numpy() / wd.n).tolist(),
            "tank_methane_rel_err": e_ch4.tolist(),
            "roofline": {"bound": "mfma", "achieved": mlp_flop / (fwd_ms / 1e3) / 1e12,
                         "peak": 2500.0, "unit": "TFLOP/s",
                         "frac": mlp_flop / (fwd_ms / 1e3) / 2.5e15,
                         "kernel": "k_mlp_fwd (BF16 MFMA forward)", "avg_launch_ms": fwd_ms},
            "final_state_rel_err_median": torch.quantile(rel, 0.5, dim=1).tolist(),
            "final_state_rel_err_p99": torch.quantile(rel, 0.99, dim=1).tolist(),
            "audit": audit}),
        "gate_tradeoff": gate_rows,
        "exact_every_R_steps": resync_rows,
        "at_stated_error": next(
            ({"tol_ion": g["tol_ion"], "tol_closure": g["tol_closure"],
              "exact_every_R_steps": g.get("period"),
              "particle_steps_per_s": g["particle_steps_per_s"],
              "speedup_vs_fp64": g["speedup_vs_fp64"], "speedup_vs_fair": g["speedup_vs_fair"],
              "criteria": "fastest surrogate setting (gate, or exact step every R steps) with "
                          "tank methane flow within 1e-3 at every step and pH within 1e-3 "
                          "(p99)"}
             for g in sorted(gate_rows + resync_rows, key=lambda r: -r["particle_steps_per_s"])
             if g["meets_1e-3"]), None),
        "fp64_rtol_sweep": sweep,
        "fair_baseline": None if fair is None else
        {"rtol": fair["rtol"], "particle_steps_per_s": fair["particle_steps_per_s"],
         "criteria": "loosest FP64 rtol with tank methane flow (every step) and pH (p99) "
                     "within 1e-3 of the rtol-1e-8 run"},
        "advection_seconds": adv_s,
    }
    del pos_k
    torch.cuda.empty_cache()
    return res


def surrogate_main(args):
    """Gated surrogate against the FP64 path on the digester field: train the
    network on integrator transitions (or load --checkpoint), then compare
    both paths (field_comparison) over --steps coupling steps."""
    import torch

    from paper_2311_08927_amd import adm1 as A
    from paper_2311_08927_amd import surrogate as S
    from paper_2311_08927_amd import workloads as W
    torch.cuda.set_device(0)
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    n_train = W.pad_ld(((1 << 24) + args.train_steps - 1) // args.train_steps, 64)
    ld_max = max(W.pad_ld(args.n), n_train)
    ctx = A.Context(ld_max, rtol=args.rtol, atol=W.atol_vector(args.rtol), variant=args.variant)
    # the surrogate's own context: its fallback integrations run at
    # --fallback-rtol (the path's error budget is 1e-3)
    ctx_fb = A.Context(ld_max, rtol=args.fallback_rtol, atol=W.atol_vector(args.fallback_rtol),
                       variant=args.variant)
    sur = S.Surrogate(ctx_fb, ld_max, 8192)
    if args.checkpoint:
        params, norm, rec = S.load_checkpoint(args.checkpoint)
        sur.set_weights(params, norm)
        rec = dict(rec, loaded_from=os.path.relpath(args.checkpoint, ROOT))
    else:
        rec = S.train_on_transitions(ctx, sur, args.train_data, 1 << 24, args.train_steps,
                                     args.train_epochs, args.train_seed, args.gas_weight,
                                     bool(args.calibrate), log)
    gates = [(args.gate_ion, args.gate_closure)] + [
        tuple(float(v) for v in g.split(":")) for g in args.gate_sweep.split(",") if g.strip()]
    fair = [float(r) for r in args.fair_rtols.split(",") if r.strip()]
    res = field_comparison(args, args.n, args.steps, sur, ctx, log, gates, fair)
    K = args.steps
    s0 = res["surrogate"]
    out = {
        "metric": "ADM1 particle-steps/sec (FP64 integrator vs gated surrogate) at stated error",
        "value": s0["particle_steps_per_s"], "unit": "particle-steps/s",
        "n_gpus": 1, "steps": K, "warmup": args.burn_in, "ms_per_step": s0["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16+f64", "data": "synthetic",
        "config": {"workload": res["workload"], "path": "gated surrogate",
                   "gate": {"tol_ion": args.gate_ion, "tol_closure": args.gate_closure},
                   "fallback_rtol": args.fallback_rtol},
        "roofline": s0["roofline"],
        "detail": dict(res, train=rec),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
