#!/usr/bin/env python3
"""Benchmark of the SALT bandflux hot path on one MI355X.

A step is one pass of the whole hot path over the 4,096-supernova batch
(~450k observations, 6 bands, uneven light curves): bandflux of every
observation, chi-square against noisy data, and the hand-written adjoint giving
d chi2 / d(z, t0, x0, x1, c) per supernova (one fused launch).  `value` is
observations evaluated per second (forward + adjoint) with all inputs resident
in HBM, over K steps launched as replays of a HIP graph; the kernel's own
duration comes from HIP events around eager launches.  Extra legs report the forward-only kernel, the broadcast sweep
(1,048,576 parameter samples x 120 observations, one observation table broadcast to
every sample) against the plain kernel on the
same work, the 65,536 x 100 forward + adjoint batch, and the fit server under
Poisson load (p50/p99 latency).  The FP64 oracle is timed on the host cores on a
bounded sample as `cpu_baseline`.

Prints one JSON line on stdout.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "bandflux evals/s (fwd, fwd+adjoint) vs FP64 err; p50/p99 fit latency"
CLOCK_SETTLE_S = 0.2       # seconds of untimed launches before the main leg's warm-up steps
PEAK_FP32_TFLOPS = 157.3       # MI355X vector FP32 (packed)
PEAK_FP32_UNPACKED_TFLOPS = 78.6   # without packed FP32, which the build disables: the attainable VALU ceiling
PEAK_HBM_GBS = 8000.0

# Algorithmic work per unit of the implemented algorithm (flops, an FMA counts 2):
#   per quadrature point of a (supernova, band): grid coordinate 4, colour law 8 (VJP 14),
#     exp 1, weight factors 1 (VJP 5), fraction 1 ........................ FWD 15, VJP 25
#   per (point, tap) pair gathered into the weight vectors: tap weight 5, one FMA per
#     weight vector (VJP: 4, plus the difference weight 4) ................ FWD 7, VJP 17
#   per (surface row, window column) of the row projections: FWD 2 FMA = 4; VJP: the
#     combined node (1 FMA), the wavelength and phase first differences (1 each) and 6 FMA
#     into the five projections = 16
#   per observation: phase coordinate 4, weights 10, taps 8 (VJP 40), partials and
#     cotangent (VJP 30) .................................................. FWD 24, VJP 90
W_PT = {"fwd": 15, "vjp": 25}
W_TAP = {"fwd": 7, "vjp": 17}
W_CELL = {"fwd": 4, "vjp": 16}
W_OBS = {"fwd": 24, "vjp": 90}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ----------------------------------------------------------------------------- work model

def group_stats(batch, lam_grids, model):
    """(points, columns, rows, observations) summed over the (supernova, band) groups of a batch,
    formed the way the kernels form them (float32 grid coordinates)."""
    f32 = np.float32
    z = batch.z.astype(f32)
    s = f32(1.0) / (f32(1.0) + z)
    n_s = np.diff(batch.sn_offsets)
    sn_of = np.repeat(np.arange(batch.n_sn), n_s)
    p = (batch.t - batch.t0[sn_of]) * s[sn_of]
    u = (p - f32(model.phase0)) * f32(1.0 / model.dphase)
    inside = (u >= 0) & (u <= model.n_phase - 1)
    a = np.clip(np.floor(np.where(inside, u, 0)), 0, model.n_phase - 2).astype(np.int64)
    edge = (a == 0) | (a == model.n_phase - 2)
    r0 = np.where(edge, a, a - 1)
    r1 = np.where(edge, a + 1, a + 2)
    tot = dict(points=0, cols=0, cells=0, obs=int(inside.sum()), groups=0)
    nb = len(lam_grids)
    key = sn_of[inside] * nb + batch.band[inside]
    if key.size == 0:
        return tot
    order = np.argsort(key, kind="stable")
    k_sorted = key[order]
    starts = np.r_[0, np.nonzero(np.diff(k_sorted))[0] + 1]
    keys = k_sorted[starts]
    rlo = np.minimum.reduceat(r0[inside][order], starts)
    rhi = np.maximum.reduceat(r1[inside][order], starts)
    sn_g = keys // nb
    b_g = keys % nb
    inv_dw = f32(1.0 / model.dwave)
    for b in range(nb):
        m = b_g == b
        if not m.any():
            continue
        lam = lam_grids[b]
        sg = s[sn_g[m]]
        v_lo = (f32(lam[0]) * sg - f32(model.wave0)) * inv_dw
        v_hi = (f32(lam[-1]) * sg - f32(model.wave0)) * inv_dw
        j0f = np.clip(np.floor(v_lo), 0, model.n_wave - 2)
        j0l = np.clip(np.floor(v_hi), 0, model.n_wave - 2)
        J = np.minimum(j0l + 2, model.n_wave - 1) - np.maximum(j0f - 1, 0) + 1
        H = rhi[m] - rlo[m] + 1
        tot["points"] += int(m.sum()) * len(lam)
        tot["cols"] += int(J.sum())
        tot["cells"] += int((J * H).sum())
        tot["groups"] += int(m.sum())
    return tot


def algorithmic_flops(st, mode):
    return (W_PT[mode] * st["points"] + 4 * W_TAP[mode] * st["points"] + W_CELL[mode] * st["cells"]
            + W_OBS[mode] * st["obs"])


def reference_flops(st, mode):
    """Direct (unfactorised) count per observation: 16 J + 40 N forward, 40 J + 90 N adjoint,
    with each group's J and N spread over its observations."""
    if st["groups"] == 0:
        return 0.0
    mean_J = st["cols"] / st["groups"]
    mean_N = st["points"] / st["groups"]
    per = (16 * mean_J + 40 * mean_N) if mode == "fwd" else (40 * mean_J + 90 * mean_N)
    return per * st["obs"]


# ----------------------------------------------------------------------------- CPU baseline (oracle)

_OR = None
_LIMITS = None
CPU_WORKERS_MAX = 16   # the host CPU share of one GPU on the GPU machines, whatever os.cpu_count() reports


def _init_worker():
    """One BLAS / OpenMP thread per worker process, so `cores` counts the threads in use."""
    global _LIMITS
    from threadpoolctl import threadpool_limits
    _LIMITS = threadpool_limits(1)


def _oracle_chunk(args):
    kind, batch, data, w = args
    if kind == "fwd":
        return _OR[6].bandflux(batch).shape[0]
    return _OR[6].chi2_grad(batch, data, w)[1].shape[0]


def _oracle_fit(args):
    from oracle.fit64 import FitOracle
    batch, z, theta0, data, w = args
    return FitOracle(_OR[6]).fit(batch, z, theta0, data, w)["chi2"]


def host_cpu():
    """CPU model and counts of the host the baseline runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "affinity_cpus": aff}


def _timed_passes(pool, work, budget_s, n_per_pass):
    """Full passes of work over the pool until budget_s seconds are spent: (items done, seconds)."""
    passes = 0
    t0 = time.perf_counter()
    while True:
        for _ in pool.imap_unordered(_oracle_chunk, work):
            pass
        passes += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    return passes * n_per_pass, time.perf_counter() - t0, passes


def cpu_baseline(batch, truth, model, bands, budget_s):
    """The FP64 oracle on the host cores, one single-threaded worker process per core (at most the
    GPU's CPU share): the metric's workload (chi-square gradient of the 4,096-supernova batch, full
    passes for about budget_s seconds) as `value`, and beside it the one-supernova call, the
    forward pass of the same batch, 200 fits of the serving workload and a 16,384-sample subset of
    the sweep."""
    global _OR
    import multiprocessing as mp

    import oracle
    _OR = {6: oracle.Oracle(model, bands)}
    host = host_cpu()
    cores = max(1, min(CPU_WORKERS_MAX, host["affinity_cpus"]))
    chunk = 16
    n_chunks = (batch.n_sn + chunk - 1) // chunk
    subs = [batch.subset(np.arange(c * chunk, min(batch.n_sn, (c + 1) * chunk))) for c in range(n_chunks)]
    tsubs = [truth.subset(np.arange(c * chunk, min(truth.n_sn, (c + 1) * chunk))) for c in range(n_chunks)]
    grad_work = [("grad", sb, np.zeros(sb.n_obs), np.ones(sb.n_obs)) for sb in subs]
    fwd_work = [("fwd", sb, None, None) for sb in tsubs]
    legs = {}
    ctx = mp.get_context("fork")
    pool = ctx.Pool(cores, initializer=_init_worker)
    try:
        done, dt, passes = _timed_passes(pool, grad_work, budget_s, batch.n_obs)
        value = done / dt
        sample = (f"FP64 oracle forward+adjoint (chi2 gradient), {passes} full passes over the {batch.n_sn} "
                  f"supernovae ({batch.n_obs} observations each pass) in {dt:.1f} s, {cores} single-threaded "
                  f"worker processes")
        done, dt, passes = _timed_passes(pool, fwd_work, 0.2 * budget_s, truth.n_obs)
        legs["fwd_4096sn"] = {"value": done / dt, "unit": "evals/s",
                              "sample": f"forward only, {passes} full passes over the batch in {dt:.1f} s"}
        # 200 fits of the serving workload (50 LM iterations each), noise-free starts as in the bench leg
        reqs = synth.fit_requests(200, k=4)
        jobs = []
        for r in reqs:
            n = len(r.t)
            b1 = synth.Batch(np.float32([r.z]), np.float32([r.theta_true[0]]), np.float32([r.theta_true[1]]),
                             np.float32([r.theta_true[2]]), np.float32([r.theta_true[3]]), r.t, r.band,
                             np.int32([0, n]))
            f = _OR[6].bandflux(b1)
            d, _, w = synth.make_data(f, [0, n], r.normals)
            jobs.append((b1, r.z, r.theta_init, d, w))
        t0 = time.perf_counter()
        pool.map(_oracle_fit, jobs, chunksize=1)
        dt = time.perf_counter() - t0
        legs["fits_200"] = {"value": len(jobs) / dt, "unit": "fits/s",
                            "sample": f"200 requests of the serving workload, FP64 LM fits of 50 iterations, "
                                      f"in {dt:.1f} s"}
        # the sweep: a 16,384-sample subset of the 1,048,576 samples, 120 observations each
        sw = synth.sweep_120_obs(n_samples=16384)
        smp, no = sw.samples, len(sw.obs_t)
        sw_work = []
        for lo in range(0, smp.n_sn, 256):
            idx = np.arange(lo, min(smp.n_sn, lo + 256))
            m = len(idx)
            sw_work.append(("fwd", synth.Batch(smp.z[idx], smp.t0[idx], smp.x0[idx], smp.x1[idx], smp.c[idx],
                                               np.tile(sw.obs_t, m), np.tile(sw.obs_band, m),
                                               np.arange(0, (m + 1) * no, no, dtype=np.int32)), None, None))
        t0 = time.perf_counter()
        for _ in pool.imap_unordered(_oracle_chunk, sw_work):
            pass
        dt = time.perf_counter() - t0
        legs["sweep_subset"] = {"value": smp.n_sn * no / dt, "unit": "evals/s",
                                "sample": f"subset: {smp.n_sn} of the 1,048,576 samples x {no} observations "
                                          f"in {dt:.1f} s"}
    finally:
        pool.close()
        pool.join()
    # one supernova, 40 observations in 4 bands: one call on one core
    o4 = oracle.Oracle(model, synth.make_bands(4))
    b1 = synth.one_sn_40_obs()
    o4.bandflux(b1)
    t0 = time.perf_counter()
    for _ in range(50):
        o4.bandflux(b1)
    legs["one_sn_40_obs"] = {"value": (time.perf_counter() - t0) / 50 * 1e6, "unit": "us per call",
                             "sample": "50 calls of the forward pass on one core"}
    return {"value": value, "unit": "evals/s", "cores": cores, "kind": "oracle", "sample": sample,
            "host": host, "legs": legs}


def _cpu_baseline_child(conn, batch, truth, model, bands, budget_s):
    conn.send(cpu_baseline(batch, truth, model, bands, budget_s))
    conn.close()


def cpu_baseline_isolated(batch, truth, model, bands, budget_s):
    """cpu_baseline in a child process that has exited (with its workers and any BLAS threads) before
    this process touches the GPU, so no host load is left behind for the timed GPU legs."""
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    rx, tx = ctx.Pipe(duplex=False)
    proc = ctx.Process(target=_cpu_baseline_child, args=(tx, batch, truth, model, bands, budget_s))
    proc.start()
    tx.close()
    res = rx.recv()
    proc.join()
    return res


# ----------------------------------------------------------------------------- HBM traffic from counters

PROFILE_VJP = os.path.join(ROOT, "profiles", "k_band_vjp_4096sn.md")


def code_only(text):
    """C/C++ source without comments, trailing spaces and blank lines."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip())


def kernel_sources_sha256():
    """Hash of the device sources' code (kernels and the headers they include; comments do not
    count, so a profile stays valid across comment edits)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2504_08081_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            with open(os.path.join(d, f), encoding="utf-8") as fh:
                h.update(code_only(fh.read()).encode())
    return h.hexdigest()


def profile_record(path):
    """The machine-readable lines of a committed rocprofv3 summary (HBM bytes and executed FP32 flops
    per launch), or {} if there is none or the kernels have changed since it was taken."""
    if not os.path.exists(path):
        return {}
    rec = {}
    with open(path) as fh:
        for line in fh:
            k, _, v = line.partition(":")
            if k.strip() in ("kernel_sources_sha256", "traffic_bytes_per_launch", "executed_fp32_flops_per_launch"):
                rec[k.strip()] = v.strip()
    if rec.get("kernel_sources_sha256") != kernel_sources_sha256():
        return {}
    out = {}
    if "traffic_bytes_per_launch" in rec:
        out["traffic"] = int(rec["traffic_bytes_per_launch"])
    if "executed_fp32_flops_per_launch" in rec:
        out["executed_flops"] = float(rec["executed_fp32_flops_per_launch"])
    return out


# ----------------------------------------------------------------------------- timing helpers

def time_launches(torch, fn, steps, warmup):
    """Per-launch HIP-event durations (ms) and the wall time of `steps` back-to-back launches."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    durs = np.array([a.elapsed_time(b) for a, b in ev])
    return durs, wall


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--sweep-samples", type=int, default=1 << 20)
    ap.add_argument("--legs", default="one,fwd,sweep,big,serve,fitbatch,nested,peaks")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device copy of this size (for calibrating HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (supernovae, sweep "
              "samples and fits are independent and would shard across GPUs with no exchange).",
              file=sys.stderr)
        sys.exit(2)
    legs = set(x for x in args.legs.split(",") if x)

    model = synth.make_model()
    bands = synth.make_bands(6)
    truth = synth.batch_4096_sn()
    ev_params = synth.perturb(truth)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: FP64 oracle on the host cores ...")
        cpu = cpu_baseline_isolated(ev_params, truth, model, bands, args.cpu_seconds)
        log(f"cpu baseline: {cpu['value']:.0f} evals/s on {cpu['cores']} cores")

    import torch
    from paper_2504_08081_amd import saltbf
    torch.cuda.set_device(0)
    ctx = saltbf.Context.from_model(model, bands)
    lam_grids = [saltbf.band_grid(b.wave, b.trans)[0] for b in bands]
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()

    def dev_batch(b):
        return dict(z=dv(b.z), t0=dv(b.t0), x0=dv(b.x0), x1=dv(b.x1), c=dv(b.c), t=dv(b.t), band=dv(b.band),
                    sn_offsets=dv(b.sn_offsets))

    # noisy data from the GPU forward model at the true parameters (timing inputs)
    dtrue = dev_batch(truth)
    f_true = ctx.bandflux(**dtrue).cpu().numpy()
    data, _, w = synth.make_data(f_true, truth.sn_offsets, synth.noise_draws(truth.n_obs))
    D = dev_batch(ev_params)
    D["data"], D["inv_sigma2"] = dv(data), dv(w)
    ctx.device_check()
    n_obs = truth.n_obs

    grad = torch.empty((truth.n_sn, 5), device="cuda")
    # the step runs on a stream of its own, so that it can be captured in a HIP graph
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    step = ctx.prepare_bandflux_vjp(**D, chi2=True, grad=grad, stream=side)
    log(f"main leg: fused forward+adjoint, {truth.n_sn} SN, {n_obs} obs, {args.steps} steps")
    # the main leg is the first GPU work of the run: 0.2 s of the same launch first brings the
    # GPU from idle to its working clocks, then the W warm-up steps
    with torch.cuda.stream(side):
        t_settle = time.perf_counter()
        while time.perf_counter() - t_settle < CLOCK_SETTLE_S:
            for _ in range(50):
                step()
            torch.cuda.synchronize()
        for _ in range(args.warmup):
            step()
    torch.cuda.synchronize()
    # (1) per-launch kernel durations: HIP events on the launch stream around each eager launch
    t0 = time.perf_counter()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for a, b in evs:
        a.record(side)
        step()
        b.record(side)
    torch.cuda.synchronize()
    wall_eager = time.perf_counter() - t0
    durs = np.array([a.elapsed_time(b) for a, b in evs])
    # (2) whole-job throughput: the K steps as replays of a graph of G launches, so that the
    #     host's launch rate does not bound it
    G = 10 if args.steps % 10 == 0 else 1
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        for _ in range(G):
            step()
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps // G):
        graph.replay()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.device_check()
    value = n_obs * args.steps / wall
    st = group_stats(ev_params, lam_grids, model)
    kern_s = float(durs.mean()) * 1e-3
    alg_flops = algorithmic_flops(st, "vjp")
    ref_flops = reference_flops(st, "vjp")
    prof = profile_record(PROFILE_VJP)
    if "executed_flops" in prof:
        flops, src = prof["executed_flops"], ("executed FP32 flops per launch (FMA 2, add and mul 1, 64 lanes) from "
                                              "the rocprofv3 counters of the same kernels, profiles/k_band_vjp_4096sn.md")
    else:
        flops, src = alg_flops, "implemented algorithm's flop count (no counter profile of the current kernels)"
    achieved = flops / kern_s / 1e12
    result = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "fwd+adjoint chi2 gradient, 4096 SN, uneven 20-200 obs, 6 bands",
                   "n_sn": truth.n_sn, "n_obs": n_obs, "bands": 6, "surface": "71x721", "parallelism": "none"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": prof.get("traffic"),
                     "achieved_source": src, "kernel": "k_band<VJP> + k_band_sum (one call)",
                     "kernel_ms": float(durs.mean()),
                     "kernel_ms_median": float(np.median(durs)),
                     "flops_per_launch": flops,
                     "attainable_peak_unpacked": PEAK_FP32_UNPACKED_TFLOPS,
                     "frac_of_unpacked": achieved / PEAK_FP32_UNPACKED_TFLOPS,
                     "reference_count": {"flops_per_launch": ref_flops, "tflops": ref_flops / kern_s / 1e12,
                                         "frac": ref_flops / kern_s / 1e12 / PEAK_FP32_TFLOPS,
                                         "per_obs": "40 J + 90 N (direct form, forward + adjoint)"},
                     "implemented_algorithm": {"flops_per_launch": alg_flops, "tflops": alg_flops / kern_s / 1e12},
                     "work": st},
        "kernel_evals_per_s": n_obs / kern_s,
        "timing": f"value: {args.steps} steps as {args.steps // G} replays of a HIP graph of {G} launches; "
                  "kernel_ms: HIP events around each of as many eager launches; before the warm-up steps, "
                  f"{CLOCK_SETTLE_S} s of the same launch brings the GPU from idle to its working clocks",
        "eager_evals_per_s": n_obs * args.steps / wall_eager,
    }
    log(f"main: {value:.3e} evals/s, kernel {durs.mean():.4f} ms, {achieved:.2f} TFLOP/s ({src[:40]})")

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_probe_bytes"] = n * 4
        del src, dst

    if "one" in legs:
        result["one_sn"] = one_sn_leg(torch, saltbf, model, dv)
        log(f"one_sn: {result['one_sn']}")

    if "fwd" in legs:
        d_nochi = {k: D[k] for k in ("z", "t0", "x0", "x1", "c", "t", "band", "sn_offsets")}
        out = torch.empty(n_obs, device="cuda")
        durs_f, wall_f = time_launches(torch, ctx.prepare_bandflux(**d_nochi, out=out), args.steps, args.warmup)
        kf = float(durs_f.mean()) * 1e-3
        result["fwd"] = {"evals_per_s": n_obs * args.steps / wall_f, "kernel_ms": float(durs_f.mean()),
                         "kernel_evals_per_s": n_obs / kf,
                         "algorithmic_tflops": algorithmic_flops(st, "fwd") / kf / 1e12,
                         "reference_count_tflops": reference_flops(st, "fwd") / kf / 1e12}
        log(f"fwd: {result['fwd']}")

    if "sweep" in legs:
        sw = synth.sweep_120_obs(n_samples=args.sweep_samples)
        smp = sw.samples
        no = len(sw.obs_t)
        f1 = ctx.bandflux(z=dv(np.float32([sw.theta_true[0]])), t0=dv(np.float32([sw.theta_true[1]])),
                          x0=dv(np.float32([sw.theta_true[2]])), x1=dv(np.float32([sw.theta_true[3]])),
                          c=dv(np.float32([sw.theta_true[4]])), t=dv(sw.obs_t), band=dv(sw.obs_band),
                          sn_offsets=dv(np.int32([0, no]))).cpu().numpy()
        sdata, _, sw_w = synth.make_data(f1, [0, no], synth.noise_draws(no, k=55))
        P = dict(z=dv(smp.z), t0=dv(smp.t0), x0=dv(smp.x0), x1=dv(smp.x1), c=dv(smp.c))
        t_o, b_o = dv(sw.obs_t), dv(sw.obs_band)
        chi = torch.empty(smp.n_sn, device="cuda")
        reps = 5
        D_s = {"data": dv(sdata), "w": dv(sw_w)}
        d_sw, wall_sw = time_launches(torch, ctx.prepare_bandflux(**P, t=t_o, band=b_o, broadcast=True, chi2=True,
                                                                  data=D_s["data"], inv_sigma2=D_s["w"], out=chi),
                                      reps, 1)
        chi_ps = torch.empty(smp.n_sn, device="cuda")
        d_ps, _ = time_launches(torch, ctx.prepare_bandflux(**P, t=t_o, band=b_o, broadcast="persistent", chi2=True,
                                                             data=D_s["data"], inv_sigma2=D_s["w"], out=chi_ps),
                                reps, 1)
        n = smp.n_sn
        tt, bb = t_o.repeat(n), b_o.repeat(n)
        off = torch.arange(0, (n + 1) * no, no, dtype=torch.int32, device="cuda")
        dd, ww = D_s["data"].repeat(n), D_s["w"].repeat(n)
        chi_pl = torch.empty(n, device="cuda")
        d_pl, wall_pl = time_launches(torch, ctx.prepare_bandflux(**P, t=tt, band=bb, sn_offsets=off, chi2=True,
                                                                  data=dd, inv_sigma2=ww, out=chi_pl), reps, 1)
        ctx.device_check()
        same = bool(torch.equal(chi, chi_pl)) and bool(torch.equal(chi, chi_ps))
        del tt, bb, off, dd, ww
        evals = n * no
        result["sweep"] = {"samples": n, "obs": no, "broadcast_evals_per_s": evals / (d_sw.mean() * 1e-3),
                           "persistent_evals_per_s": evals / (d_ps.mean() * 1e-3),
                           "plain_evals_per_s": evals / (d_pl.mean() * 1e-3),
                           "broadcast_ms": float(d_sw.mean()), "persistent_ms": float(d_ps.mean()),
                           "plain_ms": float(d_pl.mean()), "bitwise_equal": same}
        log(f"sweep: {result['sweep']}")

    if "big" in legs:
        big = synth.batch_65536_sn()
        Db = dev_batch(synth.perturb(big, k=7))
        fb = ctx.bandflux(**dev_batch(big)).cpu().numpy()
        bd, _, bw = synth.make_data(fb, big.sn_offsets, synth.noise_draws(big.n_obs, k=17))
        Db["data"], Db["inv_sigma2"] = dv(bd), dv(bw)
        gb = torch.empty((big.n_sn, 5), device="cuda")
        d_b, wall_b = time_launches(torch, ctx.prepare_bandflux_vjp(**Db, chi2=True, grad=gb), 10, 2)
        ctx.device_check()   # every band window of the batch was on the grid
        result["big_fwd_adj"] = {"n_sn": big.n_sn, "n_obs": big.n_obs, "kernel_ms": float(d_b.mean()),
                                 "evals_per_s": big.n_obs * 10 / wall_b}
        log(f"big: {result['big_fwd_adj']}")
        del Db

    if "serve" in legs and args.serve_seconds > 0:
        result["serving"] = serve_leg(torch, saltbf, model, bands, args.serve_seconds)
        log(f"serving: {result['serving']}")
        result["serving_lbfgsb"] = serve_leg(torch, saltbf, model, bands, args.serve_seconds,
                                             solver=saltbf.SB_SOLVER_LBFGSB)
        log(f"serving_lbfgsb: {result['serving_lbfgsb']}")

    if "nested" in legs:
        result["nested"] = nested_leg(torch, saltbf, model, bands)
        log(f"nested: {result['nested']}")

    if "fitbatch" in legs:
        result["fit_batch"] = fit_batch_leg(torch, saltbf, model, bands)
        log(f"fit_batch: {result['fit_batch']}")

    if "peaks" in legs:
        pk = peaks_leg(torch, saltbf)
        result["peaks"] = pk
        rl = result["roofline"]
        rl["measured_fp32_peak"] = pk["fma_f32_tflops"]
        rl["frac_of_measured"] = rl["achieved"] / pk["fma_f32_tflops"]
        log(f"peaks: {pk}")

    if cpu is not None:
        result["cpu_baseline"] = cpu
    ctx.close()
    print(json.dumps(result), flush=True)


def one_sn_leg(torch, saltbf, model, dv, calls=200):
    """One supernova, 40 observations in 4 bands: latency of one call, launch included (host clock
    from the call to the end of a synchronisation), forward and forward + adjoint."""
    ctx = saltbf.Context.from_model(model, synth.make_bands(4))
    b = synth.one_sn_40_obs()
    D = dict(z=dv(b.z), t0=dv(b.t0), x0=dv(b.x0), x1=dv(b.x1), c=dv(b.c), t=dv(b.t), band=dv(b.band),
             sn_offsets=dv(b.sn_offsets))
    out = torch.empty(b.n_obs, device="cuda")
    grad = torch.empty((1, 5), device="cuda")
    cot = dv(np.ones(b.n_obs, np.float32))
    res = {"n_obs": b.n_obs}
    for name, fn in (("fwd", ctx.prepare_bandflux(**D, out=out)),
                     ("fwd_adj", ctx.prepare_bandflux_vjp(**D, cotangent=cot, grad=grad, want_flux=True))):
        for _ in range(20):
            fn()
        torch.cuda.synchronize()
        lat = np.empty(calls)
        for i in range(calls):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            lat[i] = time.perf_counter() - t0
        durs, _ = time_launches(torch, fn, calls, 5)
        res[name] = {"p50_us": float(np.percentile(lat, 50) * 1e6), "p99_us": float(np.percentile(lat, 99) * 1e6),
                     "kernel_us": float(durs.mean() * 1e3)}
    ctx.device_check()
    ctx.close()
    return res


def nested_leg(torch, saltbf, model, bands, n_live=500, batch=4096):
    """One nested-sampling run (sb_nested_sampling) on the sweep's 120-observation light curve:
    four free parameters with uniform / log-uniform priors around the truth, z fixed; wall time,
    iterations, likelihood evaluations and ln Z."""
    sw = synth.sweep_120_obs(n_samples=16)
    no = len(sw.obs_t)
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    ctx = saltbf.Context.from_model(model, bands)
    z, t0, x0, x1, c = [float(v) for v in sw.theta_true]
    f = ctx.bandflux(z=dv(np.float32([z])), t0=dv(np.float32([t0])), x0=dv(np.float32([x0])),
                     x1=dv(np.float32([x1])), c=dv(np.float32([c])), t=dv(sw.obs_t), band=dv(sw.obs_band),
                     sn_offsets=dv(np.int32([0, no]))).cpu().numpy()
    data, sig, w = synth.make_data(f, [0, no], synth.noise_draws(no, k=55))
    log_norm = float(-np.sum(np.log(np.sqrt(2 * np.pi) * np.float64(sig))))
    pri = [(0, z, 0), (1, t0 - 1.0, t0 + 1.0), (2, x0 * 0.9, x0 * 1.1), (1, x1 - 0.5, x1 + 0.5), (1, c - 0.05, c + 0.05)]
    args = (pri, dv(sw.obs_t), dv(sw.obs_band), dv(np.float32(data)), dv(np.float32(w)))
    ctx.nested_sampling(*args, n_live=50, batch=batch, max_iter=100, log_norm=log_norm)   # warm-up
    t_start = time.perf_counter()
    r = ctx.nested_sampling(*args, n_live=n_live, batch=batch, seed=7, dlogz=0.01, log_norm=log_norm)
    dt = time.perf_counter() - t_start
    ctx.device_check()
    ctx.close()
    return {"n_live": n_live, "batch": batch, "seconds": dt, "iterations": int(r["n_iter"]),
            "evaluations": int(r["n_eval"]), "batches": int(r["n_batches"]), "evals_per_s": r["n_eval"] * no / dt,
            "logz": r["logz"], "logz_err": r["logz_err"]}


def fit_batch_leg(torch, saltbf, model, bands, n_fit=4096, reps=5):
    """Batch fits (sb_fit_batch) of 4,096 serving-workload light curves in one call, each solver:
    milliseconds per call (10 launches of 5 iterations) and fits per second."""
    reqs = synth.fit_requests(n_fit, k=4)
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    n_s = np.array([len(r.t) for r in reqs])
    off = np.zeros(n_fit + 1, np.int32)
    off[1:] = np.cumsum(n_s)
    th = np.array([r.theta_true for r in reqs])
    ti = np.array([r.theta_init for r in reqs])
    zz = np.float32([r.z for r in reqs])
    t, band = dv(np.float32(np.concatenate([r.t for r in reqs]))), dv(np.int32(np.concatenate([r.band for r in reqs])))
    res = {"n_fit": n_fit, "n_obs": int(off[-1])}
    for name, solver in (("lm", saltbf.SB_SOLVER_LM), ("lbfgsb", saltbf.SB_SOLVER_LBFGSB)):
        ctx = saltbf.Context.from_model(model, bands, solver=solver)
        f = ctx.bandflux(z=dv(zz), t0=dv(np.float32(th[:, 0])), x0=dv(np.float32(th[:, 1])),
                         x1=dv(np.float32(th[:, 2])), c=dv(np.float32(th[:, 3])), t=t, band=band,
                         sn_offsets=dv(off)).cpu().numpy()
        data, _, w = synth.make_data(f, off, np.concatenate([r.normals for r in reqs]))
        args = dict(z=dv(zz), t0=dv(np.float32(ti[:, 0])), x0=dv(np.float32(ti[:, 1])), x1=dv(np.float32(ti[:, 2])),
                    c=dv(np.float32(ti[:, 3])), t=t, band=band, fit_offsets=dv(off), data=dv(data), inv_sigma2=dv(w))
        out = torch.empty((n_fit, saltbf.FIT_OUT_WORDS), dtype=torch.int32, device="cuda")
        durs, _ = time_launches(torch, lambda: ctx.fit_batch(**args, out=out), reps, 1)
        ctx.device_check()
        r = saltbf.fit_results(out)
        res[name] = {"ms_per_call": float(durs.mean()), "fits_per_s": n_fit / (durs.mean() * 1e-3),
                     "ok": int(np.sum(r["status"] == 0)), "mean_evaluations": float(r["iters"].mean())}
        ctx.close()
    return res


def peaks_leg(torch, saltbf, reps=10):
    """The roofline denominators measured on this GPU by the library's peak probes (sb_peak_probe):
    unpacked FP32 FMA rate (TFLOP/s), conflict-free 128-bit LDS read bandwidth (TB/s) and device copy
    bandwidth (GB/s, read + write bytes), each the best of `reps` HIP-event-timed launches."""
    n_wg = 2048                                   # eight 256-thread workgroups per CU
    dst = torch.empty(n_wg * saltbf.PROBE_THREADS, device="cuda")
    out = {}
    for name, kind, iters, scale in (("fma_f32_tflops", saltbf.SB_PROBE_FMA_F32, 2048, 1e-12),
                                     ("lds_read_tbs", saltbf.SB_PROBE_LDS_READ, 512, 1e-12)):
        work = saltbf.peak_probe(kind, n_wg, iters, dst=dst)
        durs, _ = time_launches(torch, lambda: saltbf.peak_probe(kind, n_wg, iters, dst=dst), reps, 2)
        out[name] = work / (float(durs.min()) * 1e-3) * scale
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, device="cuda")
    cdst = torch.empty_like(src)
    work = saltbf.peak_probe(saltbf.SB_PROBE_COPY, nbytes, src=src, dst=cdst)
    durs, _ = time_launches(torch, lambda: saltbf.peak_probe(saltbf.SB_PROBE_COPY, nbytes, src=src, dst=cdst), reps, 2)
    out["hbm_copy_gbs"] = work / (float(durs.min()) * 1e-3) * 1e-9
    out["datasheet"] = {"fp32_vector_tflops_packed": PEAK_FP32_TFLOPS, "hbm_gbs": PEAK_HBM_GBS}
    del src, cdst
    return out


def serve_leg(torch, saltbf, model, bands, seconds, **config):
    """Poisson arrivals at 2,000 req/s: submit each request at its arrival time, collect p50/p99.
    config: sb_config overrides for the serving context."""
    rate = 2000.0
    n_req = int(rate * (seconds + 1.0))   # a 1 s warm-up, then the measured seconds
    reqs = synth.fit_requests(n_req, rate=rate)
    ctx = saltbf.Context.from_model(model, bands, **config)
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    # true fluxes of every request in one batched forward call
    n_s = np.array([len(r.t) for r in reqs])
    off = np.zeros(n_req + 1, np.int32)
    off[1:] = np.cumsum(n_s)
    th = np.array([r.theta_true for r in reqs])
    zz = np.float32([r.z for r in reqs])
    f = ctx.bandflux(z=dv(zz), t0=dv(np.float32(th[:, 0])), x0=dv(np.float32(th[:, 1])),
                     x1=dv(np.float32(th[:, 2])), c=dv(np.float32(th[:, 3])),
                     t=dv(np.concatenate([r.t for r in reqs])), band=dv(np.concatenate([r.band for r in reqs])),
                     sn_offsets=dv(off)).cpu().numpy()
    normals = np.concatenate([r.normals for r in reqs])
    data, sig, _ = synth.make_data(f, off, normals)
    tickets = []
    # the library stamps t_submit / t_admit / t_done with the monotonic clock, which time.monotonic reads
    t_start = time.monotonic()
    for i, r in enumerate(reqs):
        target = t_start + r.arrival
        while True:
            now = time.monotonic()
            if now >= target:
                break
            if target - now > 2e-4:
                time.sleep(target - now - 1e-4)
        lo, hi = off[i], off[i + 1]
        tickets.append(ctx.fit_submit(r.t, r.band, data[lo:hi], sig[lo:hi], r.z, *r.theta_init))
    res = [ctx.fit_wait(tk, 30.0) for tk in tickets]
    stats = ctx.stats()
    ctx.close()
    warm = int(1.0 * rate)
    meas = [(x, t_start + r.arrival) for x, r in zip(res[warm:], reqs[warm:]) if x is not None]
    # latency from the scheduled Poisson arrival (includes any delay before the submit call)
    lat = np.array([x.t_done - arr for x, arr in meas]) * 1e3
    lat_sub = np.array([x.t_done - x.t_submit for x, _ in meas]) * 1e3
    lag = np.array([x.t_submit - arr for x, arr in meas]) * 1e3
    queue = np.array([(x.t_admit - x.t_submit) for x, _ in meas]) * 1e3
    done = [x for x in res if x is not None]
    span = max(x.t_done for x in done) - min(x.t_submit for x in done)
    ok = sum(1 for x in done if x.status == 0)
    return {"solver": "lbfgsb" if config.get("solver") == saltbf.SB_SOLVER_LBFGSB else "lm",
            "requests": n_req, "rate_req_s": rate, "completed_ok": ok, "fits_per_s": len(done) / span,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "latency_from": "scheduled arrival",
            "submit_p50_ms": float(np.percentile(lat_sub, 50)), "submit_p99_ms": float(np.percentile(lat_sub, 99)),
            "submit_lag_p99_ms": float(np.percentile(lag, 99)),
            "mean_queue_ms": float(queue.mean()), "ticks": stats["ticks"],
            "mean_active_slots_per_tick": stats["slot_ticks"] / max(1, stats["ticks"])}


if __name__ == "__main__":
    main()
