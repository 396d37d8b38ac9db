"""Surrogate pipeline on one GPU: Monte Carlo labels -> ensemble training ->
design sweep with Monte Carlo fallback.

Every numerical step runs in libfos_mc (optics, walk, fractions, features,
training, prediction, gate, compaction, reductions); this module only
orchestrates the calls and moves device tensors around.
"""
from __future__ import annotations

import os
import time

import numpy as np

from . import fos
from . import workloads as W


def device_problem(arrays, device="cuda"):
    """MCProblem from a dict of numpy arrays (item_geometry() layout plus
    mu_s, mu_a, g)."""
    I = len(arrays["n_layers"])
    return fos.MCProblem.from_numpy(device, arrays["n_layers"], np.asarray(arrays["mu_s"]).reshape(I, -1),
                                    np.asarray(arrays["mu_a"]).reshape(I, -1), np.asarray(arrays["g"]).reshape(I, -1),
                                    np.asarray(arrays["n_layer"]).reshape(I, -1),
                                    np.asarray(arrays["thickness"]).reshape(I, -1), arrays["n_upper"],
                                    arrays["n_lower"], arrays["k_lower"], arrays["mu0"],
                                    np.asarray(arrays["photons"]).astype(np.int64))


def optics_problem(ctx, wl, device="cuda"):
    """GPU effective-medium optics of a workload, then its transport problem."""
    import torch
    req = W.optics_request(wl)
    op = fos.OpticsProblem.from_request(req, device)
    C = op.n_cells
    mus, mua, g = (torch.zeros(C, dtype=torch.float32, device=device) for _ in range(3))
    fos.fos_optics_run(ctx, op, mus, mua, g)
    geo = W.item_geometry(wl)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)
    ph = t(geo["photons"].astype(np.int64), np.int64)
    if hasattr(torch, "uint64"):
        ph = ph.view(torch.uint64)
    return fos.MCProblem(t(geo["n_layers"], np.int32), mus, mua, g, t(geo["n_layer"], np.float32).reshape(-1),
                         t(geo["thickness"], np.float32).reshape(-1), t(geo["n_upper"], np.float32),
                         t(geo["n_lower"], np.float32), t(geo["k_lower"], np.float32), t(geo["mu0"], np.float32), ph)


def paint_problem(ctx, sweep, device="cuda"):
    """Transport problem of a PaintSweep: the optics of every (design,
    wavelength) cell by fos_optics_lognormal, the other per-item arrays by
    repeating each design's values over its wavelengths."""
    import torch
    D, L = sweep.n_designs, len(sweep.wavelengths)
    n = D * L
    dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)
    lp = fos.LognormalProblem(**sweep.lognormal_tables(), species=dev(sweep.species, np.int32),
                              matrix=dev(sweep.matrix, np.int32), rmed=dev(sweep.rmed, np.int32),
                              f=dev(sweep.f, np.float64))
    mus, mua, g = (torch.empty(n, dtype=torch.float32, device=device) for _ in range(3))
    fos.fos_optics_lognormal(ctx, lp, mus, mua, g)
    per_item = lambda a: dev(a, np.float32).repeat_interleave(L)
    ph = torch.full((n,), sweep.photons, dtype=torch.int64, device=device)
    if hasattr(torch, "uint64"):
        ph = ph.view(torch.uint64)
    ones = torch.ones(n, dtype=torch.float32, device=device)
    return fos.MCProblem(torch.ones(n, dtype=torch.int32, device=device), mus, mua, g,
                         per_item(W.PAINT_NM[sweep.matrix]), per_item(sweep.thickness), ones, ones.clone(),
                         torch.zeros(n, dtype=torch.float32, device=device), ones.clone(), ph)


def take_items(prob, idx):
    """The sub-problem of the items `idx` (device int64 tensor), in that order."""
    import torch
    T = prob.tensors
    L = prob.max_layers
    rows = lambda t: t.view(prob.n_items, L)[idx].reshape(-1).contiguous()
    ph = T["photons"].view(torch.int64)[idx].contiguous().view(T["photons"].dtype)
    return fos.MCProblem(T["n_layers"][idx].contiguous(), rows(T["mu_s"]), rows(T["mu_a"]), rows(T["g"]),
                         rows(T["n_layer"]), rows(T["thickness"]), T["n_upper"][idx].contiguous(),
                         T["n_lower"][idx].contiguous(), T["k_lower"][idx].contiguous(), T["mu0"][idx].contiguous(),
                         ph)


def with_photons(prob, photons: int):
    """The same problem with every item's photon budget replaced."""
    import torch
    T = dict(prob.tensors)
    ph = torch.full((prob.n_items,), photons, dtype=torch.int64, device=T["photons"].device)
    if hasattr(torch, "uint64"):
        ph = ph.view(torch.uint64)
    T["photons"] = ph
    return fos.MCProblem(**T)


def mc_fractions(ctx, prob, seed: int, launch=None, stream=None):
    """Run the walk on every item; returns (rat [n*3] device, photon-steps,
    capped photons, largest capped fraction of an item)."""
    import torch
    n = prob.n_items
    tal = torch.zeros(n * fos.N_TALLY, dtype=torch.int64, device="cuda")
    fos.fos_mc_run(ctx, prob, seed, tal, launch=launch, stream=stream)
    rat = torch.zeros(n * 3, dtype=torch.float32, device="cuda")
    fos.fos_mc_fractions(ctx, tal, rat, stream=stream)
    t = tal.view(n, fos.N_TALLY)
    photons = t[:, :5].sum(1).clamp(min=1).double()
    capped_frac = float((t[:, 4].double() / photons).max().item()) if n else 0.0
    return rat, int(t[:, 5].sum().item()), int(t[:, 4].sum().item()), capped_frac


def training_recipe_id(seed: int, n: int) -> str:
    """Fingerprint of the training-item recipe (the first 1000 items drawn
    from `seed`) and of the labelling order and launches of n items: stored
    with saved labels, so labels are never re-joined to features drawn or
    walked by a different recipe."""
    import hashlib
    a = W.surrogate_training_items(1000, seed)
    h = hashlib.sha1()
    for k in sorted(a):
        h.update(np.ascontiguousarray(a[k]).tobytes())
    h.update(np.ascontiguousarray(_walk_cost(a)).tobytes())
    h.update(repr(label_launch_sizes(n)).encode())
    return h.hexdigest()[:16]


def _walk_cost(a):
    """Ordering key for the labelling walks of single-layer items: the
    number of scatterings of their longest walks.  A photon that diffuses
    across a slab of scattering depth tau_s needs about (tau_s (1 - g))^2
    transport mean free paths of 1 / (1 - g) scatterings each, i.e. about
    tau_s^2 (1 - g) scatterings; absorption ends a walk after about
    tau_s / tau_a of them, whichever comes first; at least one."""
    t = a["thickness"][:, 0]
    tau_s, tau_a = a["mu_s"][:, 0] * t, a["mu_a"][:, 0] * t
    diffusion = np.maximum(tau_s * tau_s * (1.0 - a["g"][:, 0]), 1.0)
    return np.minimum(tau_s / np.maximum(tau_a, 1e-12), diffusion)


def label_launch_sizes(n: int, first: int = 1024, largest: int = 262_144):
    """Items per labelling launch, longest walks first: two launches of
    `first` items, then sizes doubling every two launches up to `largest`.
    The thick items, whose walks hold most of the photon-steps, run in short
    launches; the light bulk runs in large ones."""
    sizes, size, done = [], first, 0
    while done < n:
        for _ in range(2):
            m = min(size, n - done)
            if m > 0:
                sizes.append(m)
                done += m
        size = min(2 * size, largest)
    return sizes


# photons of an item that the per-photon step cap may stop before the labels
# are rejected (a capped photon is counted in no outcome)
MAX_CAPPED_FRACTION = 1e-3


def label_stream(j: int, in_flight: int) -> int:
    """Stream of the j-th labelling launch: the first (the longest walks)
    has stream 0 to itself, the others take turns on streams 1..in_flight-1
    (with one stream, everything runs on it)."""
    if j == 0 or in_flight == 1:
        return 0
    return 1 + (j - 1) % (in_flight - 1)


def make_training_set(ctx, n: int, photons: int, seed: int, chunk: int = 125_000, log=None, label: bool = True,
                      launch=None, launch_sizes=None, launches=None, y=None, on_launch=None, in_flight: int = 2):
    """n single-layer items labelled by the walk at `photons` each.
    Returns (x [n*8], y [n*3], photon-steps, seconds).  With label=False only
    the features are made (y is None): the items are a function of
    (n, seed, chunk), so stored labels can be re-joined to their features.

    The items are ordered by _walk_cost, longest first, and walked in the
    launches of `launch_sizes` (default label_launch_sizes(n)), launch c
    under seed + c.  Every launch is prepared and queued up front, on
    `in_flight` streams: the first launch on a stream of its own, the others
    taking turns on the rest, so that a launch starts on the CUs that the
    ones before it free while their last long walks run.  Labels depend on
    (n, seed,
    chunk) and on that order and those sizes.  A label whose item had more
    than MAX_CAPPED_FRACTION of its photons stopped by the step cap raises.

    `launches` (a range of launch indices, default all) walks only those
    launches, writing their rows of `y` (a device tensor [n*3] to continue,
    or None for a new one); `on_launch(c, steps, capped)` is called as each
    launch completes, so a long labelling can be resumed."""
    import torch
    t0 = time.perf_counter()
    parts, xs = [], []
    for c, b in enumerate(range(0, n, chunk)):
        m = min(chunk, n - b)
        arrays = W.surrogate_training_items(m, seed + 7919 * c, photons=photons)
        x = torch.zeros(m * fos.SUR_FEATURES, dtype=torch.float32, device="cuda")
        fos.fos_sur_features(ctx, device_problem(arrays), x)
        xs.append(x)
        parts.append(arrays)
    x = torch.cat(xs)
    if not label:
        torch.cuda.synchronize()
        return x, None, 0, time.perf_counter() - t0
    items = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
    order = np.argsort(-_walk_cost(items), kind="stable")
    if y is None:
        y = torch.zeros(n * 3, dtype=torch.float32, device="cuda")
    if in_flight < 1:
        raise ValueError("in_flight must be >= 1")
    sizes = list(launch_sizes) if launch_sizes is not None else label_launch_sizes(n)
    if sum(sizes) != n or min(sizes) < 1:
        raise ValueError("launch sizes must be positive and add up to n")
    todo = list(range(len(sizes)) if launches is None else launches)
    starts = np.concatenate([[0], np.cumsum(sizes)])
    totals = {"steps": 0, "capped": 0, "worst_capped": 0.0}
    extra, jobs = [], []
    try:
        # Everything the walks need goes to the device first, while it is
        # idle: a copy or small kernel issued while persistent walks fill the
        # CUs waits for a free wave slot, for tens of seconds at times.  Each
        # launch has a context of its own, prepared here.
        for j, c in enumerate(todo):
            if j == 0:
                cx = ctx
            else:
                extra.append(fos.Context(0))
                cx = extra[-1].handle
            m = sizes[c]
            idx = order[starts[c]:starts[c] + m]
            prob = device_problem({k: v[idx] for k, v in items.items()})
            fos.fos_mc_prepare(cx, prob)
            jobs.append({"c": c, "ctx": cx, "m": m, "prob": prob, "idx": torch.from_numpy(idx).cuda(),
                         "tal": torch.zeros(m * fos.N_TALLY, dtype=torch.int64, device="cuda"),
                         "rat": torch.zeros(m * 3, dtype=torch.float32, device="cuda"),
                         "stats_host": torch.zeros(3, dtype=torch.float64, pin_memory=True)})
        torch.cuda.synchronize()
        # The first launch (the longest walks) has a stream of its own; the
        # others take turns on the remaining streams, each running its
        # launches back to back.  Each launch's fractions, its rows of y and
        # its counts follow its walk on its stream.
        streams = [torch.cuda.Stream() for _ in range(in_flight)]
        for j, job in enumerate(jobs):
            st = streams[label_stream(j, in_flight)]
            m = job["m"]
            with torch.cuda.stream(st):
                fos.fos_mc_execute(job["ctx"], seed + job["c"], job["tal"], launch=launch, stream=st)
                fos.fos_mc_fractions(job["ctx"], job["tal"], job["rat"], stream=st)
                y.view(n, 3)[job["idx"]] = job["rat"].view(m, 3)
                t = job["tal"].view(m, fos.N_TALLY)
                stats = torch.stack([t[:, 5].sum().double(), t[:, 4].sum().double(),
                                     (t[:, 4].double() / photons).max()])
                job["stats_host"].copy_(stats, non_blocking=True)
                job["done"] = torch.cuda.Event()
                job["done"].record(st)
        if log:
            log(f"training labels: {len(jobs)} launches queued on {in_flight} streams")
        # report each launch as it ends, in the order they end
        left = list(range(len(jobs)))
        while left:
            ended = [j for j in left if jobs[j]["done"].query()]
            for j in ended:
                job = jobs[j]
                steps, capped, worst = (float(v) for v in job["stats_host"].tolist())
                steps, capped = int(steps), int(capped)
                totals["steps"] += steps
                totals["capped"] += capped
                totals["worst_capped"] = max(totals["worst_capped"], worst)
                if log:
                    log(f"training labels: launch {job['c']} ({job['m']} items) done, {steps:.3e} photon-steps, "
                        f"{capped} capped photons (item worst {worst:.1e}), {time.perf_counter() - t0:.1f} s")
                if worst > MAX_CAPPED_FRACTION:
                    raise RuntimeError(f"labelling launch {job['c']}: an item had {worst:.2e} of its photons "
                                       f"stopped by the step cap (more than {MAX_CAPPED_FRACTION})")
                if on_launch:
                    on_launch(job["c"], steps, capped)
            left = [j for j in left if j not in ended]
            if left and not ended:
                time.sleep(0.02)
    finally:
        torch.cuda.synchronize()
        for e in extra:
            e.close()
    return x, y, totals["steps"], time.perf_counter() - t0


def train(ctx, x, y, epochs=30, batch=8192, lr=1e-3, lr_min=1e-5, seed=1):
    import torch
    hist = torch.zeros(epochs * fos.SUR_MEMBERS, dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    fos.fos_sur_train(ctx, x, y, epochs=epochs, batch=batch, lr=lr, lr_min=lr_min, seed=seed, loss_history=hist)
    torch.cuda.synchronize()
    return hist.cpu().numpy().reshape(epochs, fos.SUR_MEMBERS), time.perf_counter() - t0


def predict(ctx, x):
    import torch
    n = x.numel() // fos.SUR_FEATURES
    rat = torch.zeros(n * 3, device="cuda")
    spread = torch.zeros(n, device="cuda")
    ind = torch.zeros(n, dtype=torch.uint8, device="cuda")
    fos.fos_sur_predict(ctx, x, rat=rat, spread=spread, in_domain=ind)
    return rat, spread, ind


# the committed ensemble (written by `bench.py --workload surrogate_train`)
# and its provenance record beside it
MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "trained", "surrogate_ens4.fossur")


def load_model(ctx, path: str = MODEL_PATH) -> dict:
    """Load an ensemble written by the training leg (by default the committed
    one) after checking its bytes against the sha256 recorded in the .json
    beside it; returns that provenance record."""
    import hashlib
    import json
    blob = open(path, "rb").read()
    info_path = path[:-len(".fossur")] + ".json"
    info = json.load(open(info_path))
    if hashlib.sha256(blob).hexdigest() != info["sha256"]:
        raise ValueError(f"{path} does not match the digest in {info_path}")
    fos.fos_sur_load(ctx, blob)
    return info


def weights_only_blob(blob: bytes) -> bytes:
    """A fos_sur_save blob without the optimiser state: the header with its
    has-optimiser word cleared, the feature statistics and the weights."""
    import struct
    if blob[:8] != b"FOSSUR01":
        raise ValueError("not a surrogate blob")
    members, features, hidden, params, _has_opt, _step = struct.unpack("<6I", blob[8:32])
    body = blob[32:32 + 128 + 4 * members * params]
    return blob[:8] + struct.pack("<6I", members, features, hidden, params, 0, 0) + body


def errors(a, b):
    """max, mean and 99th percentile of |a - b| (flattened)."""
    d = np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)).ravel()
    return {"max": float(d.max()), "mean": float(d.mean()), "p99": float(np.quantile(d, 0.99))}
