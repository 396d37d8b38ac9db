"""Benchmark: plain GPU Monte Carlo photon transport on one MI355X.

Workload (the two-species paint slab): 500 log-spaced wavelengths
0.3-16 um, one 500 um slab of matrix 1.5 + 1e-4 i with species A (f = 0.08)
and B (f = 0.05), log-normal radii (median 0.25 um, sigma_ln 0.3, 20 bins),
air on both sides, normal incidence, 1e6 photons per wavelength.  Inputs are
synthetic (analytic material indices); the effective mu_s, mu_a, g of every
wavelength are computed on the GPU by fos_optics_run before timing.

One step = one pass of the transport hot path over the batch: fos_mc_prepare
(validation + packing of the item table) and fos_mc_execute (the persistent
walk), i.e. 5e8 photons.  The walk kernel's duration is taken with HIP
events on the stream it runs on, inside the timed region.

Prints one JSON line.  The CPU baseline is the FP64 oracle on a bounded
sample of the same workload (every 10th wavelength, fewer photons).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of one photon-step (a scattering step) in full-rate VALU
# lane-op slots: the Philox4x32-10 block (20 32x32->64 multiplies at a
# quarter of the full rate = 80 slots, 20 three-input xors = 20), four 24-bit
# uniforms (12), the free path (log + 6), geometry and the move (11), the
# albedo test (1), the Henyey-Greenstein sample (rcp + 10) and the direction
# update (sqrt + cos + 7); transcendentals count 4 slots each.
STEP_SLOTS = 160.0
# gfx950 FP32 vector peak 157.3 TFLOP/s = 256 CUs x 2.4 GHz x 128 FMA lanes;
# one full-rate VALU lane-op slot per FMA lane per cycle.
VALU_PEAK = 157.3e12 / 2.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "walk_two_species_500_traffic.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "walk_two_species_500_valu_counters.txt")
FP32_PEAK = 157.3e12      # FP32 vector FLOP/s (packed), MI355X
KERNEL_SOURCES = ["paper_2409_00165_amd/csrc/mc_kernels.hip", "paper_2409_00165_amd/csrc/fos_device.hpp"]


def kernel_hash() -> str:
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def profile_value(path: str, key: str, hash_key: str = "kernel_hash", source_hash=None):
    """A figure from a committed counter summary ("key: value" lines), or
    None when the kernel sources changed since the counters were taken (the
    summary's `hash_key` line against `source_hash`, by default the walk's
    kernel_hash())."""
    try:
        kv = dict(line.split(":", 1) for line in open(path) if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    if kv.get(hash_key, "").strip() != (kernel_hash() if source_hash is None else source_hash):
        return None
    try:
        return float(kv[key])
    except (KeyError, ValueError):
        return None


def measured_traffic():
    """HBM bytes per walk launch from the committed counter summary."""
    return profile_value(TRAFFIC_FILE, "traffic_bytes_per_launch")


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def _gpu_info(device: int = 0) -> dict:
    """Name, architecture, compute units and the peak engine / memory clocks
    the HIP runtime reports for the device."""
    import ctypes
    import torch
    p = torch.cuda.get_device_properties(device)
    info = {"name": p.name, "arch": p.gcnArchName, "compute_units": p.multi_processor_count}
    try:
        hip = ctypes.CDLL("libamdhip64.so")
        for key, attr in (("peak_clock_mhz", 5), ("memory_clock_mhz", 60)):   # hipDeviceAttribute{,Memory}ClockRate
            v = ctypes.c_int(0)
            if hip.hipDeviceGetAttribute(ctypes.byref(v), attr, device) == 0:
                info[key] = v.value / 1000.0
    except OSError:
        pass
    return info


def gpu_problem(ctx, wl, device="cuda"):
    """Optics on the GPU, then the transport problem as device tensors."""
    import torch
    from paper_2409_00165_amd import fos
    from paper_2409_00165_amd import workloads as W
    req = W.optics_request(wl)
    op = fos.OpticsProblem.from_request(req, device)
    C = op.n_cells
    mus = torch.zeros(C, dtype=torch.float32, device=device)
    mua = torch.zeros(C, dtype=torch.float32, device=device)
    g = torch.zeros(C, dtype=torch.float32, device=device)
    fos.fos_optics_run(ctx, op, mus, mua, g)
    geo = W.item_geometry(wl)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)
    ph = t(geo["photons"].astype(np.int64), np.int64)
    if hasattr(torch, "uint64"):
        ph = ph.view(torch.uint64)
    prob = fos.MCProblem(t(geo["n_layers"], np.int32), mus, mua, g, t(geo["n_layer"], np.float32).reshape(-1),
                         t(geo["thickness"], np.float32).reshape(-1), t(geo["n_upper"], np.float32),
                         t(geo["n_lower"], np.float32), t(geo["k_lower"], np.float32), t(geo["mu0"], np.float32),
                         ph)
    return prob, (mus, mua, g)


# Algorithmic work of one photon-step (a scattering step) by instruction
# class: one Philox4x32-10 block; 47 full-rate FP32/integer operations (four
# 24-bit uniforms 12, free path 6, geometry and move 11, albedo test 1,
# Henyey-Greenstein sample 10, direction update 7); and one each of log,
# reciprocal, square root and cosine.
STEP_CLASSES = {"philox": 1, "full_rate": 47, "log": 1, "rcp": 1, "sqrt": 1, "cos": 1}
FULL_RATE_FORMS = ("fma", "fmac", "mul")
ISSUE_ITERS = {"fma": 300_000, "fmac": 300_000, "mul": 300_000, "rcp": 80_000, "sqrt": 80_000, "log": 80_000,
               "cos": 80_000, "philox": 25_000}


def issue_rates(h, stream, reps: int = 3):
    """Measured throughput of each instruction form of the walk (lane
    operations per second; Philox: blocks per second), best of `reps`
    launches after a warm-up, HIP events on `stream`."""
    import torch
    from paper_2409_00165_amd import fos
    sink = torch.zeros(fos.fos_issue_threads(h), dtype=torch.float32, device="cuda")
    out = {}
    for kind, iters in ISSUE_ITERS.items():
        fos.fos_issue_run(h, kind, iters, sink, stream=stream)
        best = None
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ops = fos.fos_issue_run(h, kind, iters, sink, stream=stream)
            b.record(stream)
            b.synchronize()
            ms = a.elapsed_time(b)
            best = ms if best is None else min(best, ms)
        out[kind] = {"ops_per_launch": ops, "ms": best, "rate": ops / (best / 1e3)}
    return out


def issue_ceiling_step_time(rates) -> float:
    """Seconds per photon-step if the walk issued only its algorithmic work
    at the measured rates, one class after another (no overlap); the
    full-rate operations at the fastest measured full-rate form."""
    full = max(rates[k]["rate"] for k in FULL_RATE_FORMS)
    return sum(n / (full if k == "full_rate" else rates[k]["rate"]) for k, n in STEP_CLASSES.items())


def valu_issue_main(args):
    """The instruction-throughput leg: measured issue rates of the walk's
    instruction forms on its launch shape, and the resulting ceiling of
    photon-steps per second."""
    import torch
    from paper_2409_00165_amd import fos
    torch.cuda.set_device(0)
    ctx = fos.Context(0)
    stream = torch.cuda.current_stream()
    rates = issue_rates(ctx.handle, stream)
    t_step = issue_ceiling_step_time(rates)
    full = max(FULL_RATE_FORMS, key=lambda k: rates[k]["rate"])
    rec = {"metric": "VALU issue rate of the walk's instruction forms (lane-ops/s; Philox blocks/s)",
           "value": rates[full]["rate"], "unit": f"lane-ops/s ({full}, the fastest full-rate form)", "n_gpus": 1, "steps": 3, "warmup": 1,
           "ms_per_step": rates[full]["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32/u32", "data": "synthetic",
           "config": {"workload": "independent chains, CUs x 8 workgroups x 256 threads (the walk's launch shape)"},
           "rates": rates, "step_classes": STEP_CLASSES, "ceiling_photon_steps_per_s": 1.0 / t_step,
           "nominal_fp32_fma_lane_ops_per_s": VALU_PEAK, "gpu": _gpu_info(0)}
    ctx.close()
    print(json.dumps(rec), flush=True)
    return 0


LONE_CAPS = (30_000, 100_000)
LONE_TAILS = (-1, 16, 64)


def lone_step_main(args):
    """Latency of one photon-step on a lone lane, the step time of a launch's
    tail: 64 photons, one per wave (chunk 1), in a slab of optical thickness
    1e7 that none of them leaves before the step cap, run at two caps; the
    time difference over the cap difference is one step of one lane.  Two
    phase functions (forward-peaked g = 0.99999 and isotropic g = 0), each
    with the tail phase off (-1) and on (16 and 64 lanes)."""
    import torch
    from paper_2409_00165_amd import fos
    torch.cuda.set_device(0)
    ctx = fos.Context(0)
    h = ctx.handle
    one = lambda v: np.array([[v]], np.float64)
    out = {}
    for name, g in (("forward_g0.99999", 0.99999), ("isotropic_g0", 0.0)):
        prob = fos.MCProblem.from_numpy("cuda", np.array([1], np.int32), one(1e5), one(1e-12), one(g), one(1.0),
                                        one(100.0), np.array([1.0]), np.array([1.0]), np.array([0.0]),
                                        np.array([1.0]), np.array([64], np.int64))
        fos.fos_mc_prepare(h, prob)
        for tail in LONE_TAILS:
            res = {}
            for cap in LONE_CAPS:
                best, tal = None, None
                for _ in range(3):
                    t = torch.zeros(6, dtype=torch.int64, device="cuda")
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record()
                    fos.fos_mc_execute(h, 5, t, launch={"tail_lanes": tail, "max_steps": cap, "chunk": 1,
                                                        "refill_min": 1})
                    b.record()
                    b.synchronize()
                    ms = a.elapsed_time(b)
                    best = ms if best is None else min(best, ms)
                    tal = t.cpu().tolist()
                res[cap] = {"ms": best, "capped": tal[4], "steps": tal[5]}
            lo, hi = LONE_CAPS
            us = (res[hi]["ms"] - res[lo]["ms"]) / (hi - lo) * 1e3
            out[f"{name}/tail{tail}"] = {"us_per_step": us, "runs": {str(k): v for k, v in res.items()}}
            print(f"[bench] {name} tail_lanes {tail}: {us:.4f} us per lone step", file=sys.stderr, flush=True)
    key = "forward_g0.99999/tail16"
    rec = {"metric": "latency of one photon-step on a lone lane", "value": out[key]["us_per_step"],
           "unit": "us/step (forward-peaked, tail_lanes 16)", "n_gpus": 1, "steps": 3, "warmup": 0,
           "ms_per_step": None, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "64 photons, one per wave, slab tau 1e7 (mu_s 1e5, d 100, mu_a 1e-12, n 1), "
                                  f"caps {LONE_CAPS[0]} and {LONE_CAPS[1]}"},
           "cases": out, "gpu": _gpu_info(0)}
    ctx.close()
    print(json.dumps(rec), flush=True)
    return 0


def cpu_baseline(wl, optics_host, seconds_target: float):
    """FP64 oracle on every 10th wavelength; photons sized for ~target s."""
    import oracle
    from paper_2409_00165_amd import workloads as W
    geo = W.item_geometry(wl)
    idx = np.arange(0, wl.n_items, 10)
    mus, mua, g = (np.asarray(a, np.float64).reshape(wl.n_items, -1)[idx] for a in optics_host)
    f = lambda k: np.asarray(geo[k], np.float64)[idx]
    threads = oracle.default_threads()

    def run(n):
        t0 = time.perf_counter()
        o = oracle.walk_batch(geo["n_layers"][idx], mus, mua, g, f("n_layer"), f("thickness"), f("n_upper"),
                              f("n_lower"), f("k_lower"), f("mu0"), np.full(len(idx), n, np.uint64),
                              seed=0x0C9B, n_threads=threads)
        return o, time.perf_counter() - t0

    o, dt = run(2000)                       # calibration
    rate = max(o[:, 5].sum() / max(dt, 1e-9), 1.0)
    steps_per_photon = o[:, 5].sum() / (2000 * len(idx))
    n = int(max(2000, min(4_000_000, seconds_target * rate / (steps_per_photon * len(idx)))))
    o, dt = run(n)
    steps = float(o[:, 5].sum())
    return {"value": steps / dt, "unit": "photon-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(idx)} of {wl.n_items} wavelengths (every 10th) x {n} photons, FP64, "
                      f"{dt:.1f} s, {steps:.3e} photon-steps",
            "cpu": _cpu_model(), "photons_per_s": len(idx) * n / dt}


def sweep_main(args):
    """Batched sweep: N three-layer designs x 100 wavelengths with uneven photon
    budgets (log-uniform 1e4..1e6 per design) in one persistent launch,
    autotuned, captured once as a graph and replayed per step."""
    def say(msg):
        print(f"[bench] {msg} ({time.perf_counter() - t_start:.1f} s)", file=sys.stderr, flush=True)

    t_start = time.perf_counter()
    say("sweep start")
    import torch
    from paper_2409_00165_amd import fos
    from paper_2409_00165_amd import workloads as W
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    say("torch ready")
    wl = W.stacks_3layer(n_designs=args.designs)
    ctx = fos.Context(0)
    h = ctx.handle
    prob, _ = gpu_problem(h, wl)
    torch.cuda.synchronize()
    I = prob.n_items
    say(f"GPU optics done for {I} items")
    fos.fos_mc_prepare(h, prob)
    say("prepared")
    t0 = time.perf_counter()
    if args.launch_json:
        fos.fos_mc_set_launch(h, json.loads(args.launch_json))
        best, tune_ms = fos.fos_mc_get_launch(h).as_dict(), float("nan")
    else:
        if args.tune_cache:
            fos.fos_mc_autotune_cache(h, args.tune_cache)
        best, tune_ms = fos.fos_mc_autotune(h, seed=7)
    tune_s = time.perf_counter() - t0
    print(f"[bench] {I} items; autotuned launch {best} ({tune_ms:.2f} ms on the stratified sample, "
          f"tuning {tune_s:.1f} s)", file=sys.stderr, flush=True)
    tal = torch.zeros(I * fos.N_TALLY, dtype=torch.int64, device=dev)
    fos.fos_mc_graph_capture(h, tal)
    say("graph captured")
    for w in range(args.warmup):
        fos.fos_mc_graph_launch(h, args.seed + 1000 + w)
        torch.cuda.synchronize()
        say(f"warm-up sweep {w} done")
    stream = torch.cuda.current_stream()
    steps_total = 0.0
    walk_ms = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fos.fos_mc_graph_launch(h, args.seed + k)
        b.record(stream)
        b.synchronize()
        walk_ms.append(a.elapsed_time(b))
        steps_total += float(tal.cpu().numpy().reshape(I, fos.N_TALLY)[:, 5].sum())
        print(f"[bench] sweep step {k} {walk_ms[-1]:.1f} ms", file=sys.stderr, flush=True)
    elapsed = time.perf_counter() - t0
    photons = float(W.item_geometry(wl)["photons"].sum())
    rec = {
        "metric": "photon-steps/s (batched three-layer design sweep, uneven photon budgets)",
        "value": steps_total / (sum(walk_ms) / 1e3), "unit": "photon-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": float(np.mean(walk_ms)),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded designs, analytic materials; optics on the GPU)",
        "config": {"workload": f"stacks_3layer: {args.designs} designs x 100 wavelengths, 3 layers on a "
                               "3.5+0.01i substrate, photons log-uniform 1e4..1e6 per design",
                   "items": I, "photons_per_step": photons, "launch": best, "graph": True,
                   "tuning_seconds": tune_s, "tuning_sample_ms": tune_ms},
        "photons_per_s": photons * args.steps / (sum(walk_ms) / 1e3),
        "design_spectra_per_s": args.designs * args.steps / (sum(walk_ms) / 1e3),
        "mean_steps_per_photon": steps_total / (photons * args.steps),
        "wall_s": elapsed,
        "roofline": {"bound": "alu", "achieved": STEP_SLOTS * steps_total / (sum(walk_ms) / 1e3) / 1e12,
                     "peak": VALU_PEAK / 1e12, "unit": "Tslot/s",
                     "frac": STEP_SLOTS * steps_total / (sum(walk_ms) / 1e3) / VALU_PEAK, "traffic": None},
    }
    ctx.close()
    print(json.dumps(rec), flush=True)
    return 0


# forward FLOP of one row through one member: 2 x (8*256 + 3*256*256 + 256*3)
MLP_FORWARD_FLOP = 2 * (8 * 256 + 3 * 256 * 256 + 256 * 3)
BF16_MFMA_PEAK = 2.5e15   # dense BF16 MFMA, MI355X
TRAIN_SEED = 20240931     # training items and their walks
HELD_SEED = 777           # held-out items
HELD_N = 10_000
INIT_SEED = 5             # He initialisation and shuffles of the ensemble
MODEL_PATH = os.path.join(ROOT, "paper_2409_00165_amd", "trained", "surrogate_ens4.fossur")


def surrogate_record(h, args, say):
    """The design sweep run two ways on one GPU: surrogate + Monte Carlo
    fallback (fos_sweep_run, the committed ensemble) on `designs` single-layer
    paint designs x `lambdas` wavelengths, and plain Monte Carlo at the
    fallback budget on the first `mc_designs` of them; both against 1e6-photon
    Monte Carlo on the surrogate's top `verify_designs` designs, on as many
    random designs, and on the same random designs with their median radius
    and matrix index unsnapped (per-entry optics)."""
    import torch
    from paper_2409_00165_amd import fos
    from paper_2409_00165_amd import surrogate_pipeline as SP
    from paper_2409_00165_amd import workloads as W
    info = SP.load_model(h, args.model)
    say(f"surrogate: model {os.path.basename(args.model)} ({info['sha256'][:12]}) loaded")
    D, L, fb = args.designs_sweep, args.lambdas, args.fallback_photons
    sweep = W.paint_sweep(D, n_lambda=L, photons=fb)
    t0 = time.perf_counter()
    prob = SP.paint_problem(h, sweep)
    torch.cuda.synchronize()
    t_optics = time.perf_counter() - t0
    n = prob.n_items
    say(f"surrogate: sweep problem ready, {D} designs x {L} wavelengths ({t_optics:.2f} s of optics)")
    # plain Monte Carlo at the fallback budget on the first designs
    Dm = min(args.mc_designs, D)
    sub = SP.take_items(prob, torch.arange(Dm * L, device="cuda"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, steps_mc, _, _ = SP.mc_fractions(h, sub, 424242)
    torch.cuda.synchronize()
    t_mc = time.perf_counter() - t0
    del sub
    say(f"surrogate: plain Monte Carlo on {Dm} designs at {fb} photons, {t_mc:.2f} s")
    rat = torch.zeros(3 * n, device="cuda")
    used = torch.zeros(n, dtype=torch.uint8, device="cuda")
    spread = torch.zeros(n, device="cuda")
    fos.fos_sweep_run(h, prob, args.spread_max, fb, 515151, rat, used, spread=spread)   # warm-up
    torch.cuda.synchronize()
    t_sur = []
    for k in range(2):
        t0 = time.perf_counter()
        n_fb = fos.fos_sweep_run(h, prob, args.spread_max, fb, 515152 + k, rat, used, spread=spread)
        torch.cuda.synchronize()
        t_sur.append(time.perf_counter() - t0)
    n_spread = int((spread > args.spread_max).sum().item())
    say(f"surrogate: sweep {min(t_sur):.3f} s, {n_fb} of {n} items on Monte Carlo ({n_spread} by spread)")
    # the fused inference kernel alone, events on the stream it runs on
    xs = torch.zeros(8 * n, device="cuda")
    el = torch.zeros(n, dtype=torch.uint8, device="cuda")
    fos.fos_sur_features(h, prob, xs, el)
    pr = torch.zeros(3 * n, device="cuda")
    fos.fos_sur_predict(h, xs, eligible=el, rat=pr)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    fos.fos_sur_predict(h, xs, eligible=el, rat=pr)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_pred = ev0.elapsed_time(ev1) / 1e3
    del xs, el, pr
    pred_flop = float(MLP_FORWARD_FLOP) * 4 * n
    # ranking: solar-weighted R (5778 K Planck stand-in) + 8-13 um emittance
    lam = sweep.wavelengths
    wr = torch.from_numpy(W.planck_weights(lam, 5778.0, 0.3, 2.5).astype(np.float32)).cuda()
    we = torch.from_numpy(W.planck_weights(lam, 300.0, 8.0, 13.0).astype(np.float32)).cuda()
    red = torch.zeros(2 * D, device="cuda")
    fos.fos_spectral_reduce(h, D, L, rat, wr, we, red)
    fom = red.view(D, 2).sum(1).cpu().numpy()
    K = min(args.verify_designs, D)
    top = np.argsort(-fom)[:K]
    rnd = np.random.default_rng(3).choice(D, size=K, replace=False)
    ver = {}
    for j, (name, designs) in enumerate((("top", top), ("random", rnd))):
        items = torch.from_numpy((designs[:, None] * L + np.arange(L)[None, :]).ravel()).cuda()
        vprob = SP.take_items(prob, items)
        ref = SP.mc_fractions(h, SP.with_photons(vprob, 1_000_000), 99 + j)[0]
        plain = SP.mc_fractions(h, SP.with_photons(vprob, fb), 77 + j)[0]
        refn = ref.cpu().numpy()
        ver[name] = {"designs": int(K),
                     "surrogate_vs_1e6_mc": SP.errors(rat.view(n, 3)[items].cpu().numpy().ravel(), refn),
                     "plain_mc_vs_1e6_mc": SP.errors(plain.cpu().numpy(), refn),
                     "fallback_frac": float(used[items].float().mean().item())}
        say(f"surrogate: {name} {K} designs vs 1e6-photon Monte Carlo {ver[name]['surrogate_vs_1e6_mc']}")
    # the random designs again with median radius and matrix index as drawn
    # (not snapped to the sweep's grids): per-entry optics, same gate
    wl = W.paint_unsnapped(rnd, D, n_lambda=L, photons=fb)
    uprob = SP.optics_problem(h, wl)
    un = uprob.n_items
    urat = torch.zeros(3 * un, device="cuda")
    uused = torch.zeros(un, dtype=torch.uint8, device="cuda")
    fos.fos_sweep_run(h, uprob, args.spread_max, fb, 616161, urat, uused)
    uref = SP.mc_fractions(h, SP.with_photons(uprob, 1_000_000), 101)[0]
    ver["random_unsnapped"] = {"designs": int(K),
                               "surrogate_vs_1e6_mc": SP.errors(urat.cpu().numpy(), uref.cpu().numpy()),
                               "fallback_frac": float(uused.float().mean().item())}
    say(f"surrogate: random {K} unsnapped designs vs 1e6-photon Monte Carlo "
        f"{ver['random_unsnapped']['surrogate_vs_1e6_mc']}")
    worst = max(v["surrogate_vs_1e6_mc"]["max"] for v in ver.values())
    sps_sur = D / min(t_sur)
    sps_mc = Dm / t_mc
    return {
        "metric": "spectra/s: surrogate + Monte Carlo fallback vs plain GPU Monte Carlo (<=0.01 R/A/T error)",
        "value": sps_sur, "unit": "spectra/s",
        "config": {"workload": f"paint sweep: {D} single-layer designs x {L} wavelengths (0.3-16 um, log-spaced); "
                               f"median radius on the grid 0.05 exp(0.09 k) um ({W.PAINT_N_RMED} values), matrix "
                               f"index on {len(W.PAINT_NM)} values 1.30..1.70; spread gate {args.spread_max}, "
                               f"fallback {fb} photons; verification at 1e6 photons",
                   "items": n, "designs": D, "lambdas": L},
        "seconds": min(t_sur), "seconds_all": t_sur, "optics_seconds": t_optics,
        "plain_mc_spectra_per_s": sps_mc, "plain_mc_seconds": t_mc, "plain_mc_designs": Dm,
        "plain_mc_photons": fb, "plain_mc_photon_steps": steps_mc,
        "speedup_vs_plain_mc": sps_sur / sps_mc,
        "speedup_vs_plain_mc_scaled": {"1e4": sps_sur / (sps_mc * fb / 1e4), "1e6": sps_sur / (sps_mc * fb / 1e6)},
        "fallback_rate": n_fb / n, "fallback_by_spread": n_spread, "fallback_out_of_domain": n_fb - n_spread,
        "max_abs_error_vs_1e6_mc": worst, "verification": ver,
        "inference_roofline": {"bound": "mfma", "achieved": pred_flop / t_pred / 1e12, "peak": BF16_MFMA_PEAK / 1e12,
                               "unit": "TFLOP/s", "frac": pred_flop / t_pred / BF16_MFMA_PEAK,
                               "kernel": "fos::mlp_infer_kernel", "rows": n, "kernel_ms": 1e3 * t_pred,
                               "work_per_row_flop": 4 * MLP_FORWARD_FLOP},
        "model": {k: info[k] for k in ("file", "sha256", "command", "recipe", "samples", "photons_each", "epochs",
                                      "held_out_error") if k in info},
    }


def surrogate_train_main(args):
    """Surrogate training pipeline: walk-labelled training set (single
    layers, inputs log-uniform over the workloads' optical depths,
    `train_photons` each), 4-member ensemble training on the GPU, held-out
    error against Monte Carlo; writes the weights (no optimiser state) and
    their provenance to --save-model (default: the committed model path)."""
    t_start = time.perf_counter()

    def say(msg):
        print(f"[bench] {msg} ({time.perf_counter() - t_start:.1f} s)", file=sys.stderr, flush=True)

    # the labelling launches in flight each take a stream: give the process
    # that many hardware queues (HIP reads this when it starts, below), so
    # that their kernels do not wait behind each other in a shared queue
    if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < args.label_in_flight:
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(args.label_in_flight, 32))
    import hashlib
    import torch
    from paper_2409_00165_amd import fos
    from paper_2409_00165_amd import surrogate_pipeline as SP
    torch.cuda.set_device(0)
    ctx = fos.Context(0)
    h = ctx.handle
    say("surrogate training pipeline start")
    launch = {k: v for k, v in (("tail_lanes", args.tail_lanes), ("regroup_lanes", args.regroup_lanes)) if v}
    if args.launch:
        launch.update(json.loads(args.launch))
    launch = launch or None
    n_tr = args.train_samples
    if args.load_data:
        # stored labels, re-joined to features regenerated from the same item seeds
        z = np.load(args.load_data)
        if str(z["recipe"]) != SP.training_recipe_id(TRAIN_SEED, int(z["n"])):
            raise SystemExit(f"{args.load_data}: labels were drawn by another training-item recipe")
        n_tr, ph = int(z["n"]), int(z["photons"])
        x, _, _, _ = SP.make_training_set(h, n_tr, ph, seed=TRAIN_SEED, label=False)
        y = torch.from_numpy(z["y"]).cuda()
        rec = {k: z[k].item() for k in ("label_seconds", "label_photon_steps") if k in z}
        rec.update({"samples": n_tr, "photons_each": ph, "labels": f"loaded from {os.path.basename(args.load_data)}"})
        say(f"training set loaded: {n_tr} samples")
    else:
        # labels, resumable: --label-state keeps the finished launches' rows
        sizes = SP.label_launch_sizes(n_tr)
        recipe = SP.training_recipe_id(TRAIN_SEED, n_tr)
        st = {"done": [], "steps": 0, "capped": 0, "seconds": 0.0, "launch_seconds": {}}
        y = torch.zeros(n_tr * 3, dtype=torch.float32, device="cuda")
        if args.label_state and os.path.exists(args.label_state):
            z = np.load(args.label_state)
            if str(z["recipe"]) != recipe or int(z["photons"]) != args.train_photons:
                raise SystemExit(f"{args.label_state}: labels of another recipe")
            st = json.loads(str(z["state"]))
            y = torch.from_numpy(z["y"]).cuda()
            say(f"label state: launches {sorted(st['done'])} already walked")
        todo = [c for c in range(len(sizes)) if c not in st["done"]]
        if args.label_launches:
            a, b = (int(v) for v in args.label_launches.split(":"))
            todo = [c for c in todo if a <= c < b]
        t_call = time.perf_counter()

        def on_launch(c, steps, capped):
            st["done"].append(c)
            st["steps"] += steps
            st["capped"] += capped
            st["launch_seconds"][str(c)] = round(time.perf_counter() - t_call, 1)
            if args.label_state:
                np.savez(args.label_state, y=y.cpu().numpy(), recipe=recipe, photons=args.train_photons,
                         state=json.dumps(dict(st, seconds=st["seconds"] + time.perf_counter() - t_call)))

        x, y, steps, secs = SP.make_training_set(h, n_tr, args.train_photons, seed=TRAIN_SEED, log=say,
                                                 launch=launch, launches=todo, y=y, on_launch=on_launch,
                                                 in_flight=args.label_in_flight)
        st["seconds"] += secs
        if len(st["done"]) < len(sizes):
            left = [c for c in range(len(sizes)) if c not in st["done"]]
            print(json.dumps({"metric": "surrogate labels (partial)", "value": len(st["done"]), "unit": "launches",
                              "left": left, "state": args.label_state, "seconds": secs}), flush=True)
            ctx.close()
            return 0
        rec = {"samples": n_tr, "photons_each": args.train_photons, "label_seconds": st["seconds"],
               "label_photon_steps": st["steps"], "label_photon_steps_per_s": st["steps"] / st["seconds"],
               "label_capped_photons": st["capped"], "label_launches": len(sizes),
               "label_launch": launch or "default", "label_in_flight": args.label_in_flight,
               "label_launch_seconds": st["launch_seconds"]}
        say(f"labels: {n_tr} items x {args.train_photons} photons in {st['seconds']:.1f} s of walks, "
            f"{st['steps']:.3e} photon-steps, {st['capped']} capped photons")
        if args.labels_only:
            line = {"metric": "surrogate training labels (walk only)", "value": st["seconds"], "unit": "s",
                    "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": 1e3 * st["seconds"],
                    "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32 walk",
                    "data": "synthetic",
                    "config": {"workload": f"{n_tr} single-layer training items x {args.train_photons} photons, "
                                           f"longest first in {len(sizes)} launches, {args.label_in_flight} "
                                           "in flight"},
                    "labels": rec, "label_checksum": float(y.double().sum().item()),
                    "wall_s": time.perf_counter() - t_start}
            ctx.close()
            print(json.dumps(line), flush=True)
            return 0
    xh, yh, _, _ = SP.make_training_set(h, HELD_N, rec["photons_each"], seed=HELD_SEED, chunk=HELD_N, launch=launch)
    if args.save_data:
        np.savez(args.save_data, y=y.cpu().numpy(), yh=yh.cpu().numpy(), n=n_tr,
                 recipe=SP.training_recipe_id(TRAIN_SEED, n_tr), photons=rec["photons_each"],
                 label_seconds=rec.get("label_seconds", 0.0), label_photon_steps=rec.get("label_photon_steps", 0))
        say(f"training and held-out labels written to {args.save_data}")
    hist, tsec = SP.train(h, x, y, epochs=args.epochs, batch=args.batch, lr=args.lr, lr_min=args.lr * 1e-2,
                          seed=INIT_SEED)
    rec.update({"epochs": args.epochs, "batch": args.batch, "lr": args.lr, "lr_min": args.lr * 1e-2,
                "init_seed": INIT_SEED, "train_seconds": tsec, "loss_first_epoch": hist[0].tolist(),
                "loss_last_epoch": hist[-1].tolist()})
    say(f"trained {args.epochs} epochs in {tsec:.1f} s; mean loss {hist[0].mean():.4f} -> {hist[-1].mean():.4f}")
    rh, sh, ih = SP.predict(h, xh)
    torch.cuda.synchronize()
    rec["held_out_error"] = SP.errors(rh.cpu().numpy(), yh.cpu().numpy())
    rec["held_out_in_gate"] = float(((sh <= args.spread_max) & ih.bool()).float().mean().item())
    say(f"held-out ({HELD_N} items) error vs Monte Carlo {rec['held_out_error']}")
    blob = SP.weights_only_blob(fos.fos_sur_save(h))
    out = args.save_model or MODEL_PATH
    if not out.endswith(".fossur"):
        raise SystemExit("--save-model must name a .fossur file")
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    open(out, "wb").write(blob)
    info = {"file": os.path.basename(out), "sha256": hashlib.sha256(blob).hexdigest(),
            "command": "python bench.py --workload surrogate_train" +
                       (f" --tail-lanes {args.tail_lanes}" if args.tail_lanes else "") +
                       (f" --train-samples {n_tr}" if n_tr != 2_000_000 else "") +
                       (f" --train-photons {rec['photons_each']}" if rec["photons_each"] != 100_000 else "") +
                       (f" --epochs {args.epochs}" if args.epochs != 60 else ""),
            "train_seed": TRAIN_SEED, "held_out_seed": HELD_SEED, "held_out_items": HELD_N,
            "recipe": SP.training_recipe_id(TRAIN_SEED, n_tr), **rec}
    json.dump(info, open(out[:-len(".fossur")] + ".json", "w"), indent=1)
    say(f"model written to {out}")
    line = {"metric": "surrogate training pipeline (labels + training + held-out error)",
            "value": rec.get("label_seconds", 0.0) + tsec, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": 1e3 * (rec.get("label_seconds", 0.0) + tsec), "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "bf16 MFMA / f32 walk", "data": "synthetic",
            "config": {"workload": f"{n_tr} walk-labelled items x {rec['photons_each']} photons, 4 x MLP "
                                   "8-256x4-3, 60 epochs"}, "model": info, "wall_s": time.perf_counter() - t_start}
    ctx.close()
    print(json.dumps(line), flush=True)
    return 0


def surrogate_main(args):
    """The surrogate half of the metric as its own line (see surrogate_record),
    with the FP64 oracle's network forward and Monte Carlo as CPU baseline."""
    t_start = time.perf_counter()

    def say(msg):
        print(f"[bench] {msg} ({time.perf_counter() - t_start:.1f} s)", file=sys.stderr, flush=True)

    import torch
    from paper_2409_00165_amd import fos
    from paper_2409_00165_amd import surrogate_pipeline as SP
    from paper_2409_00165_amd import workloads as W
    torch.cuda.set_device(0)
    ctx = fos.Context(0)
    h = ctx.handle
    sub = surrogate_record(h, args, say)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        from oracle import mlp as omlp
        threads = oracle.default_threads()
        L, fb = args.lambdas, args.fallback_photons
        sweep = W.paint_sweep(2, n_lambda=L, photons=fb)
        prob = SP.paint_problem(h, sweep)
        T = {k: v.cpu().numpy() for k, v in prob.tensors.items() if k != "photons"}
        f64 = lambda k: T[k].astype(np.float64)
        t0 = time.perf_counter()
        o = oracle.walk_batch(T["n_layers"], f64("mu_s"), f64("mu_a"), f64("g"), f64("n_layer"), f64("thickness"),
                              f64("n_upper"), f64("n_lower"), f64("k_lower"), f64("mu0"),
                              np.full(2 * L, fb, np.uint64), seed=0x0C9B, n_threads=threads)
        dt_mc = time.perf_counter() - t0
        stats, params, _ = fos.parse_sur_blob(fos.fos_sur_save(h))
        x = torch.zeros(8 * 2 * L, device="cuda")
        fos.fos_sur_features(h, prob, x)
        xs64 = (x.view(2 * L, 8).cpu().numpy().astype(np.float64) - stats[0]) * stats[1]
        rows = np.tile(xs64, (25, 1))
        sizes = (8, 256, 256, 256, 256, 3)
        t0 = time.perf_counter()
        for m in range(4):
            v, layers, off = params[m].astype(np.float64), [], 0
            for k_in, k_out in zip(sizes[:-1], sizes[1:]):
                layers.append((v[off:off + k_in * k_out].reshape(k_in, k_out),
                               v[off + k_in * k_out:off + k_in * k_out + k_out]))
                off += k_in * k_out + k_out
            omlp.forward(layers, rows)
        dt_nn = time.perf_counter() - t0
        cpu = {"value": 2 / dt_mc, "unit": "spectra/s", "cores": threads, "kind": "oracle",
               "sample": f"plain FP64 Monte Carlo of 2 designs x {L} wavelengths at {fb} photons ({dt_mc:.1f} s, "
                         f"{float(o[:, 5].sum()):.3e} photon-steps)",
               "mlp_forward_rows_per_s": len(rows) / dt_nn,
               "mlp_sample": f"FP64 forward of the 4 members on {len(rows)} rows ({dt_nn:.2f} s, numpy)",
               "cpu": _cpu_model()}
        say(f"cpu baseline: {cpu}")
    rec = {"metric": sub["metric"], "value": sub["value"], "unit": "spectra/s", "n_gpus": 1, "steps": 2,
           "warmup": 1, "ms_per_step": 1e3 * sub["seconds"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16 MFMA / f32 walk", "data": "synthetic", "config": sub["config"],
           "roofline": dict(sub["inference_roofline"], traffic=None), "cpu_baseline": cpu,
           **{k: v for k, v in sub.items() if k not in ("metric", "value", "unit", "config", "inference_roofline")},
           "wall_s": time.perf_counter() - t_start}
    ctx.close()
    print(json.dumps(rec), flush=True)
    return 0


def context_main(args):
    """A spectrum shaped like the paper's desktop timing example (451
    wavelengths, 200 um film at f = 0.60, 5e4 photons): the GPU walk timed over
    `steps` runs, the oracle on every 10th wavelength at the same photons."""
    t_start = time.perf_counter()

    def say(msg):
        print(f"[bench] {msg} ({time.perf_counter() - t_start:.1f} s)", file=sys.stderr, flush=True)

    import torch
    import oracle
    from paper_2409_00165_amd import fos
    from paper_2409_00165_amd import workloads as W
    torch.cuda.set_device(0)
    ctx = fos.Context(0)
    h = ctx.handle
    wl = W.paper_context_451()
    prob, optics = gpu_problem(h, wl)
    n = wl.n_items
    tal = torch.zeros(n * fos.N_TALLY, dtype=torch.int64, device="cuda")
    for _ in range(args.warmup):
        fos.fos_mc_run(h, prob, args.seed, tal)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        fos.fos_mc_run(h, prob, args.seed + k, tal)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    steps = int(tal.view(n, fos.N_TALLY)[:, 5].sum().item())
    say(f"GPU: {dt * 1e3:.1f} ms per 451-wavelength spectrum, {steps / dt:.3e} photon-steps/s")
    # oracle: every 10th wavelength at the full photon count, on all host threads
    geo = W.item_geometry(wl)
    idx = np.arange(0, n, 10)
    mus, mua, g = (t.cpu().numpy().astype(np.float64).reshape(n, -1)[idx] for t in optics)
    f = lambda k: np.asarray(geo[k], np.float64)[idx]
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    o = oracle.walk_batch(geo["n_layers"][idx], mus, mua, g, f("n_layer"), f("thickness"), f("n_upper"),
                          f("n_lower"), f("k_lower"), f("mu0"), geo["photons"][idx], seed=0x0C9B, n_threads=threads)
    dto = time.perf_counter() - t0
    o_steps = float(o[:, 5].sum())
    say(f"oracle: {len(idx)} wavelengths in {dto:.1f} s on {threads} threads")
    rec = {"metric": "seconds per 451-wavelength spectrum at 5e4 photons (paper-shaped context run)",
           "value": dt, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * dt, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic (species A in n_m = 1.5; the paper's material files are absent)",
           "config": {"workload": "paper_context_451: 451 wavelengths 0.25-2.5 um, 200 um film, f = 0.60, "
                                  "r = 0.2 um, 5e4 photons per wavelength", "items": n},
           "photon_steps_per_s": steps / dt, "mean_steps_per_photon": steps / (n * 50_000),
           "cpu_baseline": {"value": dto * n / len(idx), "unit": "s (extrapolated from every 10th wavelength)",
                            "cores": threads, "kind": "oracle", "photon_steps_per_s": o_steps / dto,
                            "sample": f"{len(idx)} of {n} wavelengths x 5e4 photons, FP64, {dto:.1f} s",
                            "cpu": _cpu_model()},
           "paper_context": "the paper reports about 28 s for a Monte Carlo spectrum at 5e4 photons on a desktop "
                            "computer (its own materials; context only, not the same inputs)",
           "wall_s": time.perf_counter() - t_start}
    ctx.close()
    print(json.dumps(rec), flush=True)
    return 0


# Algorithmic FP64 work of the Mie series, counted from the operations the
# series performs (complex multiply 6 flops, complex add 2, complex divide 12
# with the real division as one flop): per downward step of a logarithmic
# derivative D_n = n/z - 1/(D_{n+1} + n/z), 12; per upward term of a
# homogeneous sphere (psi, xi recurrences, a_n and b_n, the three sums), 134;
# a coated sphere adds 216 per term (G, T recurrences, U, V and the modified
# ratios) and two more downward recurrences.
MIE_FLOP_DOWN_STEP = 12
MIE_FLOP_TERM = 134
MIE_FLOP_TERM_COATED_EXTRA = 216
FP64_PEAK = 78.6e12


def mie_work(req):
    """(size units, series terms, algorithmic FLOP) of a flat optics request,
    with the series length and downward start of the device code."""
    lam = np.asarray(req["lam"], np.float64)
    offs = np.asarray(req["offsets"], np.int64)
    cell = np.repeat(np.arange(len(lam)), np.diff(offs))
    k0 = 2.0 * np.pi / lam[cell]
    n_m = np.asarray(req["n_m"], np.float64)[cell]
    k_m = np.asarray(req["k_m"], np.float64)[cell]
    n_p = np.asarray(req["n_p"], np.float64)
    k_p = np.asarray(req["k_p"], np.float64)
    r = np.asarray(req["r"], np.float64)
    if req.get("sd") is not None:   # the 101 diameters of each spread, positive ones only
        d = (2.0 * r)[:, None] + np.asarray(req["sd"], np.float64)[:, None] * np.linspace(-3.0, 3.0, 101)[None, :]
        keep = d > 0
        rows = np.nonzero(keep)[0]
        r = 0.5 * d[keep]
        k0, n_m, k_m, n_p, k_p = (a[rows] for a in (k0, n_m, k_m, n_p, k_p))
    mag = np.hypot(n_p, k_p)
    ay = k0 * r * mag
    coated = req.get("r_core") is not None
    if coated:
        rc = np.asarray(req["r_core"], np.float64)
        ay = np.maximum(ay, k0 * rc * np.hypot(req["n_core"], req["k_core"]))
    nn = np.ceil(2.0 + ay + 4.3 * np.cbrt(ay)).astype(np.int64) + 1
    y2 = k0 * r * mag                                   # |m2 x| at the outer radius
    nstart = np.maximum(nn, np.ceil(y2).astype(np.int64)) + 16
    flop = MIE_FLOP_TERM * nn + MIE_FLOP_DOWN_STEP * nstart
    if coated:
        flop = flop + MIE_FLOP_TERM_COATED_EXTRA * nn + 2 * MIE_FLOP_DOWN_STEP * nstart
    return len(r), int(nn.sum()), float(flop.sum())


def optics_main(args):
    """Per-entry GPU optics (Mie + effective medium, FP64) on three synthetic
    request shapes: homogeneous spheres (the headline line), hollow coated
    spheres, and 101-size Gaussian spreads.  Each is timed over `steps` calls
    of fos_optics_run (HIP events on the current stream), against the FP64
    oracle on the same request (all host threads)."""
    t_start = time.perf_counter()

    def say(msg):
        print(f"[bench] {msg} ({time.perf_counter() - t_start:.1f} s)", file=sys.stderr, flush=True)

    import torch
    import oracle
    from paper_2409_00165_amd import fos
    from paper_2409_00165_amd import workloads as W
    torch.cuda.set_device(0)
    ctx = fos.Context(0)
    h = ctx.handle
    stream = torch.cuda.current_stream()
    kinds = {}
    for kind in W.MIE_KINDS:
        req = W.mie_sweep(kind)
        op = fos.OpticsProblem.from_request(req, "cuda")
        C = op.n_cells
        outs = [torch.zeros(C, dtype=torch.float32, device="cuda") for _ in range(3)]
        for _ in range(max(args.warmup, 1)):
            fos.fos_optics_run(h, op, *outs)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            fos.fos_optics_run(h, op, *outs)
        e1.record(stream)
        torch.cuda.synchronize()
        dt = e0.elapsed_time(e1) / 1e3 / args.steps
        units, terms, flop = mie_work(req)
        rec = {"cells": C, "entries": op.n_entries, "size_units": units, "series_terms": terms,
               "seconds_per_call": dt, "units_per_s": units / dt, "terms_per_s": terms / dt,
               "algorithmic_flop": flop, "fp64_tflops": flop / dt / 1e12, "frac_fp64_peak": flop / dt / FP64_PEAK}
        say(f"{kind}: {C} cells, {units} size units, {terms} series terms: {dt * 1e3:.2f} ms per call, "
            f"{units / dt:.3e} Mie evaluations/s, {flop / dt / 1e12:.2f} TFLOP/s FP64 (algorithmic)")
        if not args.no_cpu_baseline:
            # the oracle on the whole request, all host threads
            threads = oracle.default_threads()
            t0 = time.perf_counter()
            ref = oracle.optics_batch(req, threads)
            dto = time.perf_counter() - t0
            got = torch.stack(outs, 1).cpu().numpy().astype(np.float64)
            ext = np.maximum(ref[:, 0] + ref[:, 1], 1e-300)
            rel = float((np.abs(got[:, :2] - ref[:, :2]) / ext[:, None]).max())
            rec["cpu_baseline"] = {"value": units / dto, "unit": "Mie evaluations/s", "cores": threads,
                                   "kind": "oracle", "sample": f"the whole request ({C} cells, {units} size "
                                   f"units), FP64, {dto:.2f} s", "cpu": _cpu_model()}
            rec["max_rel_error_vs_oracle"] = rel
            say(f"{kind}: oracle {units / dto:.3e} Mie evaluations/s on {threads} threads; "
                f"float outputs vs oracle, max error relative to extinction {rel:.1e}")
        kinds[kind] = rec
    head = kinds["homogeneous"]
    out = {"metric": "Mie evaluations/s (per-entry GPU optics: Mie series + effective medium, FP64)",
           "value": head["units_per_s"], "unit": "Mie evaluations/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * head["seconds_per_call"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "mie_sweep homogeneous: 2000 cells x 500 spheres (radius 0.01-2 um log-uniform, "
                                  "wavelength 0.3-16 um); also coated (2000 x 50) and 101-size spreads (2000 x 5)",
                      "items": head["entries"]},
           "roofline": {"bound": "alu", "achieved": head["fp64_tflops"], "peak": FP64_PEAK / 1e12,
                        "unit": "TFLOP/s", "frac": head["frac_fp64_peak"], "traffic": None,
                        "kernel": "fos::mie_entries (whole fos_optics_run timed)",
                        "work_per_term_flop": MIE_FLOP_TERM, "work_per_down_step_flop": MIE_FLOP_DOWN_STEP},
           "kinds": kinds, "wall_s": time.perf_counter() - t_start}
    if "cpu_baseline" in head:
        out["cpu_baseline"] = head["cpu_baseline"]
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


def weighted_main(args):
    """Analog against weighted-packet walk on the two-species 500-wavelength
    slab: throughput of each, and the efficiency of the absorptance estimate,
    1 / (variance per photon x photon-steps per photon), per wavelength."""
    t_start = time.perf_counter()

    def say(msg):
        print(f"[bench] {msg} ({time.perf_counter() - t_start:.1f} s)", file=sys.stderr, flush=True)

    import torch
    from paper_2409_00165_amd import fos
    from paper_2409_00165_amd import workloads as W
    torch.cuda.set_device(0)
    ctx = fos.Context(0)
    h = ctx.handle
    wl = W.two_species_500(photons=args.photons)
    prob, _ = gpu_problem(h, wl)
    n = wl.n_items
    N = float(args.photons)
    out = {}
    for name, nt, run in (("analog", fos.N_TALLY, fos.fos_mc_run), ("weighted", fos.N_TALLY_W, fos.fos_mc_run_weighted)):
        tal = torch.zeros(n * nt, dtype=torch.int64, device="cuda")
        for _ in range(args.warmup):
            run(h, prob, args.seed, tal)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            run(h, prob, args.seed + k, tal)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        t = tal.view(n, nt).cpu().numpy().astype(np.float64)
        if name == "analog":
            steps = t[:, 5]
            a = t[:, 2] / N
            var_a = a * (1 - a)                             # per photon
        else:
            steps = t[:, 9]
            u = fos.WEIGHT_UNIT
            a = t[:, 2] / u / N
            var_a = np.maximum(t[:, 5] / u / N - a * a, 0.0)
        out[name] = {"seconds": dt, "photon_steps_per_s": steps.sum() / dt, "steps_per_photon": steps / N,
                     "A": a, "var_A_per_photon": var_a}
        say(f"{name}: {dt * 1e3:.1f} ms per step, {steps.sum() / dt:.3e} photon-steps/s, "
            f"{steps.sum() / N / n:.1f} steps per photon")
    an, wt = out["analog"], out["weighted"]
    ok = (an["var_A_per_photon"] > 0) & (wt["var_A_per_photon"] > 0)
    eff = (an["var_A_per_photon"] * an["steps_per_photon"])[ok] / (wt["var_A_per_photon"] * wt["steps_per_photon"])[ok]
    se = np.sqrt(an["var_A_per_photon"] / N + wt["var_A_per_photon"] / N)
    z = np.abs(an["A"] - wt["A"]) / np.maximum(se, 1e-30)
    rec = {"metric": "photon-steps/s of the weighted-packet walk, and its A-estimate efficiency against the analog "
                     "walk (two-species 500-wavelength slab)",
           "value": wt["photon_steps_per_s"], "unit": "photon-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * wt["seconds"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"two_species_500, {args.photons} photons per wavelength", "items": n},
           "analog_photon_steps_per_s": an["photon_steps_per_s"],
           "steps_per_photon": {"analog": float(an["steps_per_photon"].mean()),
                                "weighted": float(wt["steps_per_photon"].mean())},
           "efficiency_weighted_over_analog_A": {"median": float(np.median(eff)), "min": float(eff.min()),
                                                 "max": float(eff.max()), "wavelengths": int(ok.sum())},
           "A_agreement_max_z": float(z.max()),
           "wall_s": time.perf_counter() - t_start}
    ctx.close()
    print(json.dumps(rec), flush=True)
    return 0


OUTPUT_SOURCES = ["paper_2409_00165_amd/csrc/output.hip"]
OUTPUT_TRAFFIC = os.path.join(ROOT, "profiles", "output_stage_1e6x200_traffic.txt")
HBM_PEAK = 8.0e12            # bytes/s, MI355X HBM3E


def output_hash() -> str:
    import hashlib
    h = hashlib.sha1()
    for f in OUTPUT_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def output_main(args):
    rec = output_record(args, args.steps, args.warmup, not args.no_cpu_baseline, args.copy_calibration)
    print(json.dumps(rec), flush=True)
    return 0


def output_record(args, steps: int, warmup: int, with_cpu: bool, calibrate: bool = False) -> dict:
    """The output stage at the design sweep's size: eq. (21) solar totals,
    the 8 - 13 um band emittance and the colour of 10^6 spectra x 200
    wavelengths, synthetic and resident in HBM, through fos_output_run.  A
    step is one run over all designs; the weights are prepared once
    beforehand.  The roofline is HBM: each design's spectrum is read once and
    its 13 outputs written once."""
    import torch
    from paper_2409_00165_amd import fos
    from paper_2409_00165_amd import workloads as W
    t_start = time.perf_counter()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if calibrate:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)     # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    D, L = args.output_designs, args.lambdas
    lam = W.grid_log(0.25, 16.0, L).astype(np.float32)
    solar, band = W.solar_standin(), (8.0, 13.0, 300.0)
    rat = W.synthetic_rat_device(torch, D, L, seed=2409)
    ctx = fos.Context(0)
    h = ctx.handle
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    avail = fos.fos_output_prepare(h, lam, solar, None, band)
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t0
    tot = torch.empty(D * 4, device=dev)
    col = torch.empty(D * 9, device=dev)
    print(f"[bench] output stage ready: {D} designs x {L} wavelengths, available {avail}", file=sys.stderr, flush=True)
    for _ in range(warmup):
        fos.fos_output_run(h, D, L, rat, tot, col, stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        fos.fos_output_run(h, D, L, rat, tot, col, stream)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [a.elapsed_time(b) for a, b in ev]
    ms = float(np.mean(launch_ms))
    bytes_per_design = L * 3 * 4 + (4 + 9) * 4
    achieved = D * bytes_per_design / (ms / 1e3)
    traffic = profile_value(OUTPUT_TRAFFIC, "traffic_bytes_per_launch", "output_hash", output_hash())
    rec = {"metric": "output stage throughput: eq. (21) solar totals, band emittance and colour per spectrum",
           "value": D * steps / wall, "unit": "spectra/s", "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": wall / steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"output_stage: {D} designs x {L} wavelengths (log grid 0.25-16 um), uniform "
                                  "R+A+T simplex draws, 5778 K solar stand-in sampled 0.28-4 um, 8-13 um band at "
                                  "300 K, colour under equal energy"},
           "available": avail, "prepare_seconds": t_prep,
           "launch_ms": {"mean": ms, "min": float(np.min(launch_ms)), "max": float(np.max(launch_ms))},
           "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK, "traffic": traffic},
           "algorithmic_bytes_per_design": bytes_per_design, "gpu": _gpu_info(0)}
    if with_cpu:
        from oracle import output as O
        n = min(D, 50_000)
        sub = rat[: n * L * 3].view(n, L, 3).cpu().numpy().astype(np.float64)
        sol64 = (solar[0].astype(np.float64), solar[1].astype(np.float64))
        done, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < args.cpu_seconds * 2.0 / 3.0:
            O.output_stage(lam.astype(np.float64), sub, sol64, None, band)
            done += n
        dt = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": done / dt, "unit": "spectra/s", "cores": 1, "kind": "oracle",
                               "sample": f"the first {n} designs, repeated for {dt:.1f} s (numpy FP64, one thread)"}
    rec["wall_s"] = time.perf_counter() - t_start
    ctx.close()
    del rat, tot, col
    torch.cuda.empty_cache()
    return rec


def main(argv=None):
    print("[bench] start", file=sys.stderr, flush=True)
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--photons", type=int, default=1_000_000)
    ap.add_argument("--seed", type=int, default=0x5EED)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch", type=str, default="",
                    help="JSON fos_mc_launch overrides (the walk of the default workload; surrogate_train: the label walks)")
    ap.add_argument("--workload", default="two_species_500",
                    choices=["two_species_500", "stacks_3layer", "surrogate", "surrogate_train", "paper_context",
                             "weighted", "optics", "valu_issue", "lone_step", "output_stage"],
                    help="two_species_500 (default, the headline line; with the surrogate sweep as a sub-record), "
                         "stacks_3layer (batched sweep), surrogate (the committed ensemble: design sweep with Monte "
                         "Carlo fallback against plain Monte Carlo), surrogate_train (walk labels + training + "
                         "held-out error; writes the model) or "
                         "paper_context (a run shaped like the paper's desktop timing, GPU and oracle) or "
                         "weighted (analog vs weighted-packet walk: throughput and A-estimate efficiency) or "
                         "optics (per-entry GPU Mie + effective medium: homogeneous, coated, spread) or "
                         "valu_issue (issue rates of the walk's instruction forms) or "
                         "lone_step (step latency of a lone lane, tail phase off and on) or "
                         "output_stage (eq. (21) totals, band emittance and colour of 10^6 spectra)")
    ap.add_argument("--train-samples", type=int, default=2_000_000)
    ap.add_argument("--train-photons", type=int, default=100_000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lambdas", type=int, default=200)
    ap.add_argument("--spread-max", type=float, default=0.01)
    ap.add_argument("--fallback-photons", type=int, default=100_000)
    ap.add_argument("--verify-designs", type=int, default=1000,
                    help="top and random designs of the sweep verified at 1e6 photons")
    ap.add_argument("--designs-sweep", type=int, default=1_000_000, help="designs of the surrogate paint sweep")
    ap.add_argument("--mc-designs", type=int, default=4096,
                    help="designs of the sweep timed with plain Monte Carlo (the first ones)")
    ap.add_argument("--no-surrogate", action="store_true", help="leave the surrogate sub-record out")
    ap.add_argument("--no-output-stage", action="store_true", help="leave the output-stage sub-record out")
    ap.add_argument("--tune-cache", default="", help="stacks_3layer: launch cache file of the autotuner")
    ap.add_argument("--launch-json", default="",
                    help="stacks_3layer: use this launch (JSON) instead of tuning")
    ap.add_argument("--tail-lanes", type=int, default=16,
                    help="label walks: tail_lanes launch knob (0 = the context default)")
    ap.add_argument("--regroup-lanes", type=int, default=32,
                    help="label walks: regroup_lanes launch knob (0 = the context default, -1 = off)")
    ap.add_argument("--label-in-flight", type=int, default=8, help="label walks: launches in flight")
    ap.add_argument("--labels-only", action="store_true",
                    help="surrogate_train: walk the labels, report their time, and stop (no training or model)")
    ap.add_argument("--label-state", default="", help="surrogate_train: resumable label state (.npz)")
    ap.add_argument("--label-launches", default="", help="surrogate_train: walk only launches a:b of the labels")
    ap.add_argument("--save-data", default="", help="write the walk-labelled training and held-out sets (.npz)")
    ap.add_argument("--load-data", default="", help="read training and held-out sets written by --save-data")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--batch", type=int, default=2048)
    ap.add_argument("--save-model", default="", help="surrogate_train: model path (default: the committed one)")
    ap.add_argument("--model", default=MODEL_PATH, help="surrogate sweep: the ensemble to load (.fossur)")
    ap.add_argument("--designs", type=int, default=4096, help="designs of the stacks_3layer sweep")
    ap.add_argument("--output-designs", type=int, default=1_000_000, help="designs of the output_stage leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB device copy first (HBM counter calibration under rocprofv3)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the transport shards by items across GPUs with one tally gather, not built here)",
              file=sys.stderr)
        return 2
    if args.workload == "surrogate":
        return surrogate_main(args)
    if args.workload == "surrogate_train":
        return surrogate_train_main(args)
    if args.workload == "valu_issue":
        return valu_issue_main(args)
    if args.workload == "lone_step":
        return lone_step_main(args)
    if args.workload == "stacks_3layer":
        return sweep_main(args)
    if args.workload == "paper_context":
        return context_main(args)
    if args.workload == "weighted":
        return weighted_main(args)
    if args.workload == "optics":
        return optics_main(args)
    if args.workload == "output_stage":
        return output_main(args)

    import torch
    from paper_2409_00165_amd import fos
    from paper_2409_00165_amd import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print("[bench] torch ready", file=sys.stderr, flush=True)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)     # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    wl = W.two_species_500(photons=args.photons)
    ctx = fos.Context(0)
    h = ctx.handle
    launch = json.loads(args.launch) if args.launch else None
    prob, optics = gpu_problem(h, wl)
    I = prob.n_items
    print(f"[bench] optics and problem ready: {I} items", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    tallies = [torch.zeros(I * fos.N_TALLY, dtype=torch.int64, device=dev) for _ in range(args.steps)]
    warm = torch.zeros(I * fos.N_TALLY, dtype=torch.int64, device=dev)
    for w in range(args.warmup):
        fos.fos_mc_run(h, prob, args.seed + 1000 + w, warm, launch=launch)
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        fos.fos_mc_prepare(h, prob)
        ev[k][0].record(stream)
        fos.fos_mc_execute(h, args.seed + k, tallies[k], launch=launch)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"[bench] timed {args.steps} steps in {elapsed:.3f} s", file=sys.stderr, flush=True)

    tal = np.stack([t.cpu().numpy().reshape(I, fos.N_TALLY) for t in tallies])
    steps_total = float(tal[:, :, 5].sum())
    photons_total = float(tal[:, :, :5].sum())
    assert photons_total == float(args.steps) * I * args.photons, "photon conservation failed"
    walk_ms = np.array([a.elapsed_time(b) for a, b in ev])
    walk_s = float(walk_ms.mean()) / 1e3
    steps_per_launch = steps_total / args.steps
    achieved = STEP_SLOTS * steps_per_launch / walk_s
    L = fos.fos_mc_get_launch(h).as_dict()
    if launch:
        L.update(launch)

    rec = {
        "metric": "photon-steps/s (plain GPU Monte Carlo, 500-wavelength two-species slab)",
        "value": steps_total / elapsed,
        "unit": "photon-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (analytic material indices; optics computed on the GPU)",
        "config": {"workload": "two_species_500: 500 wavelengths 0.3-16 um, 500 um slab, species A f=0.08 + "
                               "B f=0.05, log-normal r_med 0.25 um sigma_ln 0.3 x 20 bins, 1e6 photons/wavelength",
                   "items": I, "photons_per_item": args.photons, "launch": L},
        "photons_per_s": photons_total / elapsed,
        "spectra_per_s": args.steps / elapsed,
        "mean_steps_per_photon": steps_total / photons_total,
        "walk_kernel_ms": float(walk_ms.mean()),
        "walk_kernel_ms_median": float(np.median(walk_ms)),
        "walk_kernel_ms_all": [round(float(x), 3) for x in walk_ms],
        "seed": args.seed,
        "gpu": _gpu_info(0),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                     "unit": "Tslot/s", "frac": achieved / VALU_PEAK, "traffic": measured_traffic(),
                     "work_per_step_slots": STEP_SLOTS, "steps_per_launch": steps_per_launch,
                     "kernel": "fos::walk", "kernel_hash": kernel_hash()},
    }
    # the same walk against the measured issue rates of its own instruction
    # forms, and its FP32 arithmetic against the FP32 FLOP peak
    rates = issue_rates(h, stream)
    t_ceiling = issue_ceiling_step_time(rates)
    steps_per_s_kernel = steps_per_launch / walk_s
    rec["roofline"]["measured_issue"] = {
        "frac": steps_per_s_kernel * t_ceiling, "ceiling_photon_steps_per_s": 1.0 / t_ceiling,
        "achieved_photon_steps_per_s": steps_per_s_kernel, "step_classes": STEP_CLASSES,
        "rates": {k: v["rate"] for k, v in rates.items()},
        "note": "frac = photon-steps/s of the walk x (seconds per photon-step at the measured rates of its "
                "algorithmic instruction classes, one class after another)"}
    flop_step = profile_value(VALU_FILE, "fp32_flop_per_photon_step")
    rec["roofline"]["fp32_flop"] = None if flop_step is None else {
        "flop_per_photon_step": flop_step, "achieved": flop_step * steps_per_s_kernel / 1e12,
        "peak": FP32_PEAK / 1e12, "unit": "TFLOP/s", "frac": flop_step * steps_per_s_kernel / FP32_PEAK}
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline ...", file=sys.stderr, flush=True)
        host = [o.cpu().numpy() for o in optics]
        rec["cpu_baseline"] = cpu_baseline(wl, host, args.cpu_seconds)
        rec["gpu_over_cpu"] = rec["value"] / rec["cpu_baseline"]["value"]
    if not args.no_surrogate:
        # the metric's second half: surrogate + Monte Carlo fallback against
        # plain GPU Monte Carlo on the paint sweep, with the committed model
        del prob, optics, tallies, warm
        torch.cuda.empty_cache()
        t_sub = time.perf_counter()
        say = lambda m: print(f"[bench] {m} ({time.perf_counter() - t_sub:.1f} s)", file=sys.stderr, flush=True)
        rec["surrogate"] = surrogate_record(h, args, say)
    if not args.no_output_stage:
        # the output stage (eq. (21) totals, band emittance, colour) on 10^6 synthetic spectra
        print("[bench] output stage ...", file=sys.stderr, flush=True)
        rec["output_stage"] = output_record(args, 10, 2, False)
    ctx.close()
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
