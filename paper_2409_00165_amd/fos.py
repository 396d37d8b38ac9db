"""Python binding of libfos_mc (ctypes; argument marshalling only).

Every function has the name of the C entry point it wraps (include/fos_mc.h)
and takes torch tensors that already live on the context's GPU; PyTorch is
used only for device memory and streams.  All compute happens in the HIP
library: if ``libfos_mc.so`` is missing this module raises on first use --
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, Structure, c_char_p, c_float, c_int, c_int32, c_uint32, c_uint64, c_void_p

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfos_mc.so")

FOS_MAX_LAYERS = 8
N_TALLY = 6
TALLY_NAMES = ("r_spec", "r_diff", "absorbed", "transmitted", "capped", "steps")
N_TALLY_W = 11
TALLY_W_NAMES = ("r_spec", "r_diff", "absorbed", "transmitted", "r_diff2", "absorbed2", "transmitted2",
                 "roulette", "capped", "steps", "photons")
WEIGHT_UNIT = float(1 << 36)
STATUS = {0: "FOS_OK", 1: "FOS_E_INVALID_ARG", 2: "FOS_E_UNSUPPORTED", 3: "FOS_E_DEVICE",
          4: "FOS_E_OUT_OF_MEMORY", 5: "FOS_E_INTERNAL", 6: "FOS_E_NOT_PREPARED"}


class FosError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.status_name = STATUS.get(status, str(status))
        super().__init__(f"{self.status_name}: {message}")


class fos_mc_problem(Structure):
    _fields_ = [("n_items", c_int32), ("max_layers", c_int32), ("n_layers", c_void_p),
                ("mu_s", c_void_p), ("mu_a", c_void_p), ("g", c_void_p), ("n_layer", c_void_p),
                ("thickness", c_void_p), ("n_upper", c_void_p), ("n_lower", c_void_p),
                ("k_lower", c_void_p), ("mu0", c_void_p), ("photons", c_void_p)]


class fos_optics_problem(Structure):
    _fields_ = [("n_cells", c_int32), ("lam", c_void_p), ("n_m", c_void_p), ("k_m", c_void_p),
                ("offsets", c_void_p), ("n_p", c_void_p), ("k_p", c_void_p), ("r", c_void_p),
                ("f", c_void_p), ("sd", c_void_p), ("r_core", c_void_p), ("n_core", c_void_p),
                ("k_core", c_void_p)]


class fos_lognormal_problem(Structure):
    _fields_ = [("n_lambda", c_int32), ("lam", c_void_p), ("n_species", c_int32), ("n_p", c_void_p),
                ("k_p", c_void_p), ("n_matrix", c_int32), ("n_m", c_void_p), ("k_m", ctypes.c_double),
                ("r0", ctypes.c_double), ("dlnr", ctypes.c_double), ("n_rmed", c_int32), ("n_bins", c_int32),
                ("w", c_void_p), ("n_designs", c_int32), ("species", c_void_p), ("matrix", c_void_p),
                ("rmed", c_void_p), ("f", c_void_p)]


class fos_train_opts(Structure):
    _fields_ = [("epochs", c_int32), ("batch", c_int32), ("lr", c_float), ("lr_min", c_float),
                ("seed", c_uint64), ("resume", c_int32), ("loss_history", c_void_p)]


class fos_spectrum(Structure):
    _fields_ = [("n", c_int32), ("um", c_void_p), ("value", c_void_p)]


class fos_output_spec(Structure):
    _fields_ = [("solar", c_void_p), ("illuminant", c_void_p), ("band_lo_um", c_float), ("band_hi_um", c_float),
                ("band_temperature_k", c_float)]


OUTPUT_SOLAR, OUTPUT_BAND, OUTPUT_COLOUR = 1, 2, 4
OUTPUT_TOTALS = ("R_s", "A_s", "T_s", "band_emittance")
OUTPUT_COLOUR_NAMES = ("X", "Y", "Z", "L*", "a*", "b*", "sRGB_r", "sRGB_g", "sRGB_b")


class fos_mc_launch(Structure):
    _fields_ = [("block_size", c_int32), ("refill_min", c_int32), ("chunk", c_int32),
                ("blocks_per_cu", c_int32), ("max_steps", c_uint64), ("tail_lanes", c_int32),
                ("regroup_lanes", c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libfos_mc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2409_00165_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.fos_abi_version.restype = c_int
        L.fos_status_string.restype = c_char_p
        L.fos_status_string.argtypes = [c_int]
        L.fos_create.argtypes = [c_int, POINTER(c_void_p)]
        L.fos_create.restype = c_int
        L.fos_destroy.argtypes = [c_void_p]
        L.fos_destroy.restype = None
        L.fos_last_error.argtypes = [c_void_p]
        L.fos_last_error.restype = c_char_p
        L.fos_mc_prepare.argtypes = [c_void_p, POINTER(fos_mc_problem), c_void_p]
        L.fos_mc_prepare.restype = c_int
        L.fos_mc_execute.argtypes = [c_void_p, c_uint64, POINTER(fos_mc_launch), c_void_p, c_void_p]
        L.fos_mc_execute.restype = c_int
        L.fos_mc_run.argtypes = [c_void_p, POINTER(fos_mc_problem), c_uint64, POINTER(fos_mc_launch),
                                 c_void_p, c_void_p]
        L.fos_mc_run.restype = c_int
        L.fos_mc_run_noalloc.argtypes = [c_void_p, POINTER(fos_mc_problem), c_uint64, POINTER(fos_mc_launch),
                                         c_void_p, c_void_p]
        L.fos_mc_run_noalloc.restype = c_int
        L.fos_issue_threads.argtypes = [c_void_p]
        L.fos_issue_threads.restype = ctypes.c_int64
        L.fos_issue_run.argtypes = [c_void_p, c_int32, c_int32, c_void_p, POINTER(c_uint64), c_void_p]
        L.fos_issue_run.restype = c_int
        L.fos_mc_prepared_items.argtypes = [c_void_p]
        L.fos_mc_prepared_items.restype = c_int32
        L.fos_mc_get_launch.argtypes = [c_void_p, POINTER(fos_mc_launch)]
        L.fos_mc_get_launch.restype = c_int
        L.fos_mc_set_launch.argtypes = [c_void_p, POINTER(fos_mc_launch)]
        L.fos_mc_set_launch.restype = c_int
        L.fos_mc_autotune.argtypes = [c_void_p, c_uint64, c_uint64, POINTER(fos_mc_launch), POINTER(c_float),
                                      c_void_p]
        L.fos_mc_autotune.restype = c_int
        L.fos_mc_autotune_cache.argtypes = [c_void_p, c_char_p]
        L.fos_mc_autotune_cache.restype = c_int
        L.fos_mc_graph_capture.argtypes = [c_void_p, POINTER(fos_mc_launch), c_void_p, c_void_p]
        L.fos_mc_graph_capture.restype = c_int
        L.fos_mc_handoff_counts.argtypes = [c_void_p, POINTER(c_uint64), POINTER(c_uint64), c_void_p]
        L.fos_mc_handoff_counts.restype = c_int
        L.fos_mc_graph_launch.argtypes = [c_void_p, c_uint64, c_void_p]
        L.fos_mc_graph_launch.restype = c_int
        L.fos_sur_features.argtypes = [c_void_p, POINTER(fos_mc_problem), c_void_p, c_void_p, c_void_p]
        L.fos_sur_features.restype = c_int
        L.fos_sur_train.argtypes = [c_void_p, c_void_p, c_void_p, ctypes.c_int64, POINTER(fos_train_opts), c_void_p]
        L.fos_sur_train.restype = c_int
        L.fos_sur_predict.argtypes = [c_void_p, c_void_p, c_void_p, ctypes.c_int64, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p]
        L.fos_sur_predict.restype = c_int
        L.fos_sur_grad.argtypes = [c_void_p, c_void_p, c_void_p, ctypes.c_int64, c_void_p, c_void_p, c_void_p]
        L.fos_sur_grad.restype = c_int
        L.fos_sur_save.argtypes = [c_void_p, c_void_p, POINTER(ctypes.c_size_t)]
        L.fos_sur_save.restype = c_int
        L.fos_sur_load.argtypes = [c_void_p, c_void_p, ctypes.c_size_t]
        L.fos_sur_load.restype = c_int
        L.fos_mc_fractions.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]
        L.fos_mc_fractions.restype = c_int
        L.fos_mc_execute_weighted.argtypes = [c_void_p, c_uint64, POINTER(fos_mc_launch), c_void_p, c_void_p]
        L.fos_mc_execute_weighted.restype = c_int
        L.fos_mc_run_weighted.argtypes = [c_void_p, POINTER(fos_mc_problem), c_uint64, POINTER(fos_mc_launch),
                                          c_void_p, c_void_p]
        L.fos_mc_run_weighted.restype = c_int
        L.fos_mc_weighted_fractions.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]
        L.fos_mc_weighted_fractions.restype = c_int
        L.fos_sweep_run.argtypes = [c_void_p, POINTER(fos_mc_problem), c_float, c_uint64, c_uint64, c_void_p,
                                    c_void_p, c_void_p, POINTER(ctypes.c_int64), c_void_p]
        L.fos_sweep_run.restype = c_int
        L.fos_spectral_reduce.argtypes = [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
        L.fos_spectral_reduce.restype = c_int
        L.fos_output_prepare.argtypes = [c_void_p, c_int32, c_void_p, POINTER(fos_output_spec), POINTER(c_int32),
                                         c_void_p]
        L.fos_output_prepare.restype = c_int
        L.fos_output_run.argtypes = [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]
        L.fos_output_run.restype = c_int
        L.fos_output_weights.argtypes = [c_void_p, c_void_p, c_void_p, POINTER(c_int32), c_void_p]
        L.fos_output_weights.restype = c_int
        L.fos_optics_run.argtypes = [c_void_p, POINTER(fos_optics_problem), c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_void_p]
        L.fos_optics_run.restype = c_int
        L.fos_optics_lognormal.argtypes = [c_void_p, POINTER(fos_lognormal_problem), c_void_p, c_void_p, c_void_p,
                                           c_void_p]
        L.fos_optics_lognormal.restype = c_int
        L.fos_philox_words.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_uint64, c_void_p,
                                       c_void_p]
        L.fos_philox_words.restype = c_int
        L.fos_eval_fresnel.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                       c_void_p]
        L.fos_eval_fresnel.restype = c_int
        L.fos_eval_hg.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]
        L.fos_eval_hg.restype = c_int
        _lib = L
    return _lib


def _check(ctx, status: int):
    if status != 0:
        msg = fos_last_error(ctx) if ctx else ""
        raise FosError(status, msg)


def _stream(stream):
    if stream is None:
        import torch
        return c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return c_void_p(stream)
    return c_void_p(stream.cuda_stream)


def _ptr(t, dtype=None, n=None):
    """Device pointer of a contiguous torch tensor (checked)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libfos_mc takes device tensors")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def fos_abi_version() -> int:
    return lib().fos_abi_version()


def fos_status_string(s: int) -> str:
    return lib().fos_status_string(s).decode()


def fos_create(hip_device: int = 0):
    h = c_void_p()
    st = lib().fos_create(hip_device, ctypes.byref(h))
    if st != 0:
        raise FosError(st, f"fos_create(device={hip_device}) failed")
    return h


def fos_destroy(ctx) -> None:
    if ctx:
        lib().fos_destroy(ctx)


def fos_last_error(ctx) -> str:
    return lib().fos_last_error(ctx).decode()


class MCProblem:
    """Device tensors of one fos_mc_problem (kept alive with the struct)."""

    def __init__(self, n_layers, mu_s, mu_a, g, n_layer, thickness, n_upper, n_lower, k_lower, mu0,
                 photons):
        import torch
        self.tensors = dict(n_layers=n_layers, mu_s=mu_s, mu_a=mu_a, g=g, n_layer=n_layer,
                            thickness=thickness, n_upper=n_upper, n_lower=n_lower, k_lower=k_lower,
                            mu0=mu0, photons=photons)
        I = n_layers.numel()
        L = mu_s.numel() // max(I, 1) if I else (mu_s.shape[-1] if mu_s.dim() == 2 else 1)
        self.n_items, self.max_layers = I, L
        s = fos_mc_problem()
        s.n_items, s.max_layers = I, L
        s.n_layers = _ptr(n_layers, torch.int32, I)
        for k in ("mu_s", "mu_a", "g", "n_layer", "thickness"):
            setattr(s, k, _ptr(self.tensors[k], torch.float32, I * L))
        for k in ("n_upper", "n_lower", "k_lower", "mu0"):
            setattr(s, k, _ptr(self.tensors[k], torch.float32, I))
        s.photons = _ptr(photons, torch.uint64 if hasattr(torch, "uint64") else torch.int64, I)
        self.struct = s

    @classmethod
    def from_numpy(cls, device, n_layers, mu_s, mu_a, g, n_layer, thickness, n_upper, n_lower, k_lower,
                   mu0, photons):
        import numpy as np
        import torch

        def f32(x):
            return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(device)

        I = len(n_layers)
        L = int(np.asarray(mu_s).reshape(I, -1).shape[1]) if I else 1
        ph = torch.from_numpy(np.ascontiguousarray(photons, dtype=np.int64)).to(device)
        if hasattr(torch, "uint64"):
            ph = ph.view(torch.uint64)
        return cls(torch.from_numpy(np.ascontiguousarray(n_layers, dtype=np.int32)).to(device),
                   *[f32(np.asarray(a).reshape(I, L)) for a in (mu_s, mu_a, g, n_layer, thickness)],
                   *[f32(a) for a in (n_upper, n_lower, k_lower, mu0)], ph)


def _launch(launch):
    if launch is None:
        return None
    if isinstance(launch, fos_mc_launch):
        return ctypes.byref(launch)
    L = fos_mc_launch()
    for k, v in dict(launch).items():
        setattr(L, k, int(v))
    return ctypes.byref(L)


def fos_mc_prepare(ctx, problem: MCProblem, stream=None) -> None:
    _check(ctx, lib().fos_mc_prepare(ctx, ctypes.byref(problem.struct), _stream(stream)))


def fos_mc_execute(ctx, seed: int, tallies, launch=None, stream=None) -> None:
    import torch
    n = fos_mc_prepared_items(ctx)
    _check(ctx, lib().fos_mc_execute(ctx, c_uint64(seed), _launch(launch),
                                     _ptr(tallies, None, n * N_TALLY) if n else _ptr(tallies),
                                     _stream(stream)))


def fos_mc_run(ctx, problem: MCProblem, seed: int, tallies, launch=None, stream=None) -> None:
    _ptr(tallies, None, problem.n_items * N_TALLY)
    _check(ctx, lib().fos_mc_run(ctx, ctypes.byref(problem.struct), c_uint64(seed), _launch(launch),
                                 _ptr(tallies), _stream(stream)))


def fos_mc_run_noalloc(ctx, problem: MCProblem, seed: int, tallies, launch=None, stream=None) -> None:
    _ptr(tallies, None, problem.n_items * N_TALLY)
    _check(ctx, lib().fos_mc_run_noalloc(ctx, ctypes.byref(problem.struct), c_uint64(seed), _launch(launch),
                                         _ptr(tallies), _stream(stream)))


ISSUE_KINDS = {"fma": 0, "rcp": 1, "sqrt": 2, "log": 3, "cos": 4, "philox": 5, "fmac": 6, "mul": 7}


def fos_issue_threads(ctx) -> int:
    return lib().fos_issue_threads(ctx)


def fos_issue_run(ctx, kind: str, iters: int, sink, stream=None) -> int:
    """One launch of the instruction-throughput kernel `kind`; returns the
    lane operations (Philox: blocks) it issues."""
    import torch
    ops = c_uint64()
    _check(ctx, lib().fos_issue_run(ctx, ISSUE_KINDS[kind], iters, _ptr(sink, torch.float32, fos_issue_threads(ctx)),
                                    ctypes.byref(ops), _stream(stream)))
    return ops.value


def fos_mc_autotune(ctx, seed: int = 1, sample_photons: int = 0, stream=None):
    """Tune the launch on a stratified sample of the prepared problem;
    returns (launch dict, ms on the sample)."""
    best = fos_mc_launch()
    ms = c_float()
    _check(ctx, lib().fos_mc_autotune(ctx, c_uint64(seed), c_uint64(sample_photons), ctypes.byref(best),
                                      ctypes.byref(ms), _stream(stream)))
    return best.as_dict(), ms.value


def fos_mc_autotune_cache(ctx, path) -> None:
    _check(ctx, lib().fos_mc_autotune_cache(ctx, (path or "").encode()))


def fos_mc_graph_capture(ctx, tallies, launch=None, stream=None) -> None:
    n = fos_mc_prepared_items(ctx)
    _check(ctx, lib().fos_mc_graph_capture(ctx, _launch(launch), _ptr(tallies, None, n * N_TALLY),
                                           _stream(stream)))


def fos_mc_handoff_counts(ctx, stream=None):
    """(photons handed between waves, hand-offs lost) of the last regrouping walk."""
    handed, lost = c_uint64(0), c_uint64(0)
    _check(ctx, lib().fos_mc_handoff_counts(ctx, ctypes.byref(handed), ctypes.byref(lost), _stream(stream)))
    return int(handed.value), int(lost.value)


def fos_mc_graph_launch(ctx, seed: int, stream=None) -> None:
    _check(ctx, lib().fos_mc_graph_launch(ctx, c_uint64(seed), _stream(stream)))


def fos_mc_fractions(ctx, tallies, rat, stream=None) -> None:
    import torch
    n = tallies.numel() // N_TALLY
    _check(ctx, lib().fos_mc_fractions(ctx, n, _ptr(tallies), _ptr(rat, torch.float32, 3 * n), _stream(stream)))


def fos_mc_execute_weighted(ctx, seed: int, tallies, launch=None, stream=None) -> None:
    n = fos_mc_prepared_items(ctx)
    _check(ctx, lib().fos_mc_execute_weighted(ctx, c_uint64(seed), _launch(launch),
                                              _ptr(tallies, None, n * N_TALLY_W) if n else _ptr(tallies),
                                              _stream(stream)))


def fos_mc_run_weighted(ctx, problem: MCProblem, seed: int, tallies, launch=None, stream=None) -> None:
    _ptr(tallies, None, problem.n_items * N_TALLY_W)
    _check(ctx, lib().fos_mc_run_weighted(ctx, ctypes.byref(problem.struct), c_uint64(seed), _launch(launch),
                                          _ptr(tallies), _stream(stream)))


def fos_mc_weighted_fractions(ctx, tallies, rat, se=None, stream=None) -> None:
    import torch
    n = tallies.numel() // N_TALLY_W
    _check(ctx, lib().fos_mc_weighted_fractions(ctx, n, _ptr(tallies), _ptr(rat, torch.float32, 3 * n),
                                                _ptr(se, torch.float32, 3 * n), _stream(stream)))


def fos_mc_prepared_items(ctx) -> int:
    return lib().fos_mc_prepared_items(ctx)


def fos_mc_get_launch(ctx) -> fos_mc_launch:
    L = fos_mc_launch()
    _check(ctx, lib().fos_mc_get_launch(ctx, ctypes.byref(L)))
    return L


def fos_mc_set_launch(ctx, launch) -> None:
    _check(ctx, lib().fos_mc_set_launch(ctx, _launch(launch)))


class OpticsProblem:
    """Device tensors of one fos_optics_problem (float64 cells, CSR particles)."""

    def __init__(self, lam, n_m, k_m, offsets, n_p, k_p, r, f, sd=None, r_core=None, n_core=None, k_core=None):
        import torch
        self.tensors = dict(lam=lam, n_m=n_m, k_m=k_m, offsets=offsets, n_p=n_p, k_p=k_p, r=r, f=f, sd=sd,
                            r_core=r_core, n_core=n_core, k_core=k_core)
        C = lam.numel()
        P = n_p.numel()
        s = fos_optics_problem()
        s.n_cells = C
        for k in ("lam", "n_m", "k_m"):
            setattr(s, k, _ptr(self.tensors[k], torch.float64, C))
        s.offsets = _ptr(offsets, torch.int64, C + 1)
        for k in ("n_p", "k_p", "r", "f", "sd", "r_core", "n_core", "k_core"):
            t = self.tensors[k]
            setattr(s, k, _ptr(t, torch.float64, P) if (P and t is not None) else None)
        self.n_cells, self.n_entries, self.struct = C, P, s

    @classmethod
    def from_request(cls, req, device="cuda"):
        """From a workloads.optics_request() dict of numpy arrays (sd, r_core,
        n_core, k_core optional)."""
        import numpy as np
        import torch
        t = lambda k, dt=np.float64: (None if req.get(k) is None else
                                      torch.from_numpy(np.ascontiguousarray(req[k], dtype=dt)).to(device))
        return cls(t("lam"), t("n_m"), t("k_m"), t("offsets", np.int64), t("n_p"), t("k_p"), t("r"), t("f"),
                   t("sd"), t("r_core"), t("n_core"), t("k_core"))


class LognormalProblem:
    """One fos_lognormal_problem: the grid tables as host float64 arrays (kept
    alive here) and the per-design arrays as device tensors."""

    def __init__(self, lam, n_p, k_p, n_m, k_m, r0, dlnr, n_rmed, w, species, matrix, rmed, f):
        import numpy as np
        import torch
        h = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        self.host = dict(lam=h(lam), n_p=h(n_p), k_p=h(k_p), n_m=h(n_m), w=h(w))
        self.tensors = dict(species=species, matrix=matrix, rmed=rmed, f=f)
        L = self.host["lam"].size
        S = self.host["n_p"].size // L
        D = species.numel()
        s = fos_lognormal_problem()
        s.n_lambda, s.n_species, s.n_matrix = L, S, self.host["n_m"].size
        s.lam, s.n_p, s.k_p = (self.host[k].ctypes.data for k in ("lam", "n_p", "k_p"))
        s.n_m, s.w = self.host["n_m"].ctypes.data, self.host["w"].ctypes.data
        s.k_m, s.r0, s.dlnr, s.n_rmed, s.n_bins = float(k_m), float(r0), float(dlnr), int(n_rmed), self.host["w"].size
        s.n_designs = D
        for k in ("species", "matrix", "rmed"):
            setattr(s, k, _ptr(self.tensors[k], torch.int32, D))
        s.f = _ptr(f, torch.float64, D)
        self.n_lambda, self.n_designs, self.struct = L, D, s


def fos_optics_lognormal(ctx, problem: LognormalProblem, mu_s=None, mu_a=None, g=None, stream=None) -> None:
    import torch
    C = problem.n_designs * problem.n_lambda
    _check(ctx, lib().fos_optics_lognormal(ctx, ctypes.byref(problem.struct), _ptr(mu_s, torch.float32, C),
                                           _ptr(mu_a, torch.float32, C), _ptr(g, torch.float32, C),
                                           _stream(stream)))


def fos_optics_run(ctx, problem: OpticsProblem, mu_s=None, mu_a=None, g=None, out_f64=None,
                   stream=None) -> None:
    import torch
    C = problem.n_cells
    _check(ctx, lib().fos_optics_run(ctx, ctypes.byref(problem.struct),
                                     _ptr(mu_s, torch.float32, C), _ptr(mu_a, torch.float32, C),
                                     _ptr(g, torch.float32, C), _ptr(out_f64, torch.float64, 3 * C),
                                     _stream(stream)))


SUR_FEATURES = 8
SUR_MEMBERS = 4
SUR_PARAMS = 200451


def fos_sur_features(ctx, problem: MCProblem, x, eligible=None, stream=None) -> None:
    import torch
    n = problem.n_items
    _check(ctx, lib().fos_sur_features(ctx, ctypes.byref(problem.struct), _ptr(x, torch.float32, n * SUR_FEATURES),
                                       _ptr(eligible, torch.uint8, n), _stream(stream)))


def fos_sur_train(ctx, x, y, epochs=10, batch=8192, lr=1e-3, lr_min=1e-5, seed=1, resume=False,
                  loss_history=None, stream=None) -> None:
    import torch
    n = x.numel() // SUR_FEATURES
    o = fos_train_opts(epochs, batch, lr, lr_min, seed, 1 if resume else 0,
                       _ptr(loss_history, torch.float32, epochs * SUR_MEMBERS))
    _check(ctx, lib().fos_sur_train(ctx, _ptr(x, torch.float32, n * SUR_FEATURES), _ptr(y, torch.float32, n * 3),
                                    n, ctypes.byref(o), _stream(stream)))


def fos_sur_predict(ctx, x, eligible=None, rat=None, spread=None, in_domain=None, members=None,
                    stream=None) -> None:
    import torch
    n = x.numel() // SUR_FEATURES
    _check(ctx, lib().fos_sur_predict(ctx, _ptr(x, torch.float32, n * SUR_FEATURES), _ptr(eligible, torch.uint8, n),
                                      n, _ptr(rat, torch.float32, 3 * n), _ptr(spread, torch.float32, n),
                                      _ptr(in_domain, torch.uint8, n),
                                      _ptr(members, torch.float32, SUR_MEMBERS * 3 * n), _stream(stream)))


def fos_sur_grad(ctx, x, y, grads, loss=None, stream=None) -> None:
    import torch
    n = x.numel() // SUR_FEATURES
    _check(ctx, lib().fos_sur_grad(ctx, _ptr(x, torch.float32), _ptr(y, torch.float32, 3 * n), n,
                                   _ptr(grads, torch.float32, SUR_MEMBERS * SUR_PARAMS),
                                   _ptr(loss, torch.float32, SUR_MEMBERS), _stream(stream)))


def fos_sur_save(ctx) -> bytes:
    n = ctypes.c_size_t(0)
    _check(ctx, lib().fos_sur_save(ctx, None, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(ctx, lib().fos_sur_save(ctx, buf, ctypes.byref(n)))
    return buf.raw[:n.value]


def fos_sur_load(ctx, blob: bytes) -> None:
    _check(ctx, lib().fos_sur_load(ctx, blob, len(blob)))


def fos_sweep_run(ctx, problem: MCProblem, spread_max: float, fallback_photons: int, seed: int, rat, used_mc,
                  spread=None, stream=None) -> int:
    """Surrogate + Monte Carlo fallback for every item; returns the number of
    items that went to Monte Carlo."""
    import torch
    n = problem.n_items
    nf = ctypes.c_int64(0)
    _check(ctx, lib().fos_sweep_run(ctx, ctypes.byref(problem.struct), c_float(spread_max), c_uint64(fallback_photons),
                                    c_uint64(seed), _ptr(rat, torch.float32, 3 * n), _ptr(spread, torch.float32, n),
                                    _ptr(used_mc, torch.uint8, n), ctypes.byref(nf), _stream(stream)))
    return nf.value


def fos_spectral_reduce(ctx, designs: int, lambdas: int, rat, w_r, w_e, out, stream=None) -> None:
    import torch
    _check(ctx, lib().fos_spectral_reduce(ctx, designs, lambdas, _ptr(rat, torch.float32, designs * lambdas * 3),
                                          _ptr(w_r, torch.float32, lambdas), _ptr(w_e, torch.float32, lambdas),
                                          _ptr(out, torch.float32, 2 * designs), _stream(stream)))


def _host_f32(a):
    import numpy as np
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def fos_output_prepare(ctx, lambda_um, solar=None, illuminant=None, band=None, stream=None) -> int:
    """Prepare the output stage for the grid lambda_um (host array, um).
    solar / illuminant: (um, value) host arrays or None; band: (lo_um,
    hi_um, temperature_k) or None.  Returns the OUTPUT_* bits available."""
    lam = _host_f32(lambda_um)
    keep = [lam]

    def spectrum(sp):
        if sp is None:
            return None
        um, val = _host_f32(sp[0]), _host_f32(sp[1])
        if um.shape != val.shape:
            raise ValueError("spectrum wavelengths and values differ in length")
        keep.extend((um, val))
        st = fos_spectrum(um.size, um.ctypes.data_as(c_void_p), val.ctypes.data_as(c_void_p))
        keep.append(st)
        return ctypes.cast(ctypes.pointer(st), c_void_p)

    spec = fos_output_spec(spectrum(solar), spectrum(illuminant), *(band if band is not None else (0.0, 0.0, 0.0)))
    avail = c_int32(0)
    _check(ctx, lib().fos_output_prepare(ctx, lam.size, lam.ctypes.data_as(c_void_p), ctypes.byref(spec),
                                         ctypes.byref(avail), _stream(stream)))
    return avail.value


def fos_output_run(ctx, designs: int, lambdas: int, rat, totals, colour=None, stream=None) -> None:
    """totals [designs, 4] and colour [designs, 9] (or None) of the spectra
    rat [designs, lambdas, 3], all device float32 tensors."""
    import torch
    _check(ctx, lib().fos_output_run(ctx, designs, lambdas, _ptr(rat, torch.float32, designs * lambdas * 3),
                                     _ptr(totals, torch.float32, designs * 4),
                                     _ptr(colour, torch.float32, designs * 9), _stream(stream)))


def fos_output_weights(ctx, lambdas: int, weights=None, params=None, stream=None) -> int:
    """Copy the prepared weights [5, lambdas] and colour parameters [12]
    into device tensors; returns the OUTPUT_* bits."""
    import torch
    avail = c_int32(0)
    _check(ctx, lib().fos_output_weights(ctx, _ptr(weights, torch.float32, 5 * lambdas),
                                         _ptr(params, torch.float32, 12),
                                         ctypes.byref(avail), _stream(stream)))
    return avail.value


def parse_sur_blob(blob: bytes):
    """(stats [4, 8], params [4, SUR_PARAMS], adam_step) of a fos_sur_save blob."""
    import numpy as np
    assert blob[:8] == b"FOSSUR01"
    hdr = np.frombuffer(blob[8:32], np.uint32)
    stats = np.frombuffer(blob[32:160], np.float32).reshape(4, 8)
    P = int(hdr[0]) * int(hdr[3])
    params = np.frombuffer(blob[160:160 + 4 * P], np.float32).reshape(int(hdr[0]), int(hdr[3]))
    return stats, params, int(hdr[5])


def fos_philox_words(ctx, photon, step, stream_ids, seed: int, out, stream=None) -> None:
    n = photon.numel()
    _check(ctx, lib().fos_philox_words(ctx, n, _ptr(photon), _ptr(step), _ptr(stream_ids), c_uint64(seed),
                                       _ptr(out, None, 4 * n), _stream(stream)))


def fos_eval_fresnel(ctx, c, ni, nt, kt, out, stream=None) -> None:
    n = c.numel()
    _check(ctx, lib().fos_eval_fresnel(ctx, n, _ptr(c), _ptr(ni), _ptr(nt), _ptr(kt), _ptr(out),
                                       _stream(stream)))


def fos_eval_hg(ctx, g, u01, out, stream=None) -> None:
    n = g.numel()
    _check(ctx, lib().fos_eval_hg(ctx, n, _ptr(g), _ptr(u01), _ptr(out), _stream(stream)))


class Context:
    """RAII wrapper: ``with Context(0) as ctx: fos_mc_run(ctx.handle, ...)``."""

    def __init__(self, device: int = 0):
        self.handle = fos_create(device)

    def close(self):
        if self.handle:
            fos_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass
