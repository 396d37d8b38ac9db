"""Write the oracle's expected tallies for the GPU parity tests.

Calls only the CPU oracle (``oracle/``) and the input recipes
(``paper_2409_00165_amd.workloads``).  The optics tables are stored rounded
to float32 -- exactly the values the GPU path receives -- and the oracle
walks those same values (widened to float64).

    python tests/golden/make_oracle_golden.py [single_slab_23|two_species_500|stacks_3layer|all]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2409_00165_amd import workloads as W  # noqa: E402

ORACLE_SEED = 0x0F05_0001   # the GPU tests use other seeds: independent samples


def _problem(wl):
    mus, mua, g = oracle.workload_optics(wl)
    geo = W.item_geometry(wl)
    f32 = lambda a: np.asarray(a, dtype=np.float32)
    return dict(n_layers=geo["n_layers"].tolist(),
                mu_s=f32(mus).tolist(), mu_a=f32(mua).tolist(), g=f32(g).tolist(),
                n_layer=f32(geo["n_layer"]).tolist(), thickness=f32(geo["thickness"]).tolist(),
                n_upper=f32(geo["n_upper"]).tolist(), n_lower=f32(geo["n_lower"]).tolist(),
                k_lower=f32(geo["k_lower"]).tolist(), mu0=f32(geo["mu0"]).tolist(),
                photons=[int(x) for x in geo["photons"]])


def _walk(p, seed, items=None, photons=None):
    I = len(p["n_layers"])
    idx = np.arange(I) if items is None else np.asarray(items)
    a = {k: np.asarray(v, dtype=np.float64)[idx] for k, v in p.items()
         if k not in ("n_layers", "photons")}
    ph = np.asarray(p["photons"], dtype=np.uint64)[idx] if photons is None else \
        np.full(len(idx), photons, np.uint64)
    return oracle.walk_batch(np.asarray(p["n_layers"], np.int32)[idx], a["mu_s"], a["mu_a"], a["g"],
                             a["n_layer"], a["thickness"], a["n_upper"], a["n_lower"], a["k_lower"],
                             a["mu0"], ph, seed=seed, streams=idx.astype(np.uint32))


def stacks_stratified_designs(wl, k):
    """Indices of k designs of a stacks workload spread evenly over its
    photon budgets (sorted by budget, the designs at quantiles (j + 1/2)/k)."""
    ph = np.array([d.photons for d in wl.designs])
    order = np.argsort(ph, kind="stable")
    return order[((np.arange(k) + 0.5) * len(ph) / k).astype(int)]


def make(name: str):
    t0 = time.time()
    extra = {}
    if name == "single_slab_23":
        wl = W.single_slab_23()
        p = _problem(wl)
        items = list(range(len(p["n_layers"])))
    elif name == "two_species_500":
        wl = W.two_species_500()
        p = _problem(wl)
        items = list(range(len(p["n_layers"])))
    elif name == "stacks_3layer":
        # 64 of the 4096 benchmark designs x 100 wavelengths at their own
        # photon budgets (log-uniform 1e4..1e6), stratified over the budget
        # range: the designs at the budget quantiles (j + 1/2) / 64
        full = W.stacks_3layer(n_designs=4096)
        designs = stacks_stratified_designs(full, 64)
        wl = W.Workload("stacks_3layer", full.wavelengths, [full.designs[d] for d in designs])
        p = _problem(wl)
        items = list(range(len(p["n_layers"])))
        extra["designs"] = [int(d) for d in designs]
    else:
        raise SystemExit(f"unknown workload {name}")
    tal = _walk(p, ORACLE_SEED, items)
    out = dict(workload=name, oracle_seed=ORACLE_SEED, items=items,
               problem=p, tallies=tal.astype(np.int64).tolist(),
               note="written by tests/golden/make_oracle_golden.py (oracle only)",
               oracle_seconds=round(time.time() - t0, 1), **extra)
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"{path}: {len(items)} items, {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or ["all"]
    if names == ["all"]:
        names = ["single_slab_23", "stacks_3layer", "two_species_500"]
    for n in names:
        make(n)
