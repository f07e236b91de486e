"""Autotuner of the FMM plans: picks ncrit and the library's tunable
parameters for a point set, expansion order and precision by timing pair
evaluations (Laplace + Yukawa, potential and gradient, the step of the
direct formulation's matvec) on the device at hand, and caches the choice
per (device, precision, p, point-count range).

Tunables (fmm_set_tuning; defaults in DEFAULTS):
  tile_split2 / tile_split4   leaf tiles of at most this many targets run as
                              2 half-waves / 4 quarter-waves
  work_cap_min / work_cap_div leaf tiles with more source work than
                              max(min, total / div) are cut into parts
  far_weight                  cost of a surface source against a point source
  gemm_rbw                    16-row blocks per wave in the translation GEMMs
  m2l_factored                M2L operators split per offset by a truncated
                              SVD and applied in two passes
  pair_order                  order of the pair evaluation's near field and
                              P2L against the far-field passes (0..4)
  near_lds                    LDS bytes held per near-field wave of a pair
                              evaluation (caps its waves per compute unit)
  gemm_lat                    translation GEMM launches of at most this many
                              workgroups use the latency-bound kernel
  near_early, near_early_grid per mille of the near-field items (the
                              shortest) started at once on a small grid
                              beside the upward passes and the M2L (order 3)
  near_early_start            the early near-field items with the far-field
                              passes (0) or once P2M is done (1); searched
                              together with near_early
  m2l_early                   the two finest levels' M2L on a third side
                              stream beside the coarser M2M levels
  m2l_cols                    bf16x3 M2L columns per workgroup (64 or 128;
                              not searched: 128 halves the occupancy)
  gemm_chain                  the M2M levels, and the L2L levels, of a pair
                              evaluation in one launch each (not searched:
                              slower on every workload measured)

The search is coordinate descent: ncrit first (with the defaults), then the
work cap, the tile splits, the surface weight, the GEMM forms and the pass
order, each stage keeping the fastest value when it beats the current one by
more than 1% (the spread of repeated timings).  The tunables interact with
ncrit (the early near-field split gains most at larger leaves), so the two
fastest ncrit values each run the stages, and their final settings are timed
again side by side.  Plans built during a stage share their tree
(same ncrit and item parameters) or their operators (same ncrit) with the
live plans of the search, so a trial costs little more than its timing."""
from __future__ import annotations

import contextlib
import ctypes
import json
import math
import os
import time

import torch

from . import _lib
from ._lib import check, lib
from .fmm import FMMPlan, eval_pair

DEFAULTS = {"tile_split2": 32, "tile_split4": 16, "work_cap_min": 512, "work_cap_div": 16384, "far_weight": 1.15,
            "gemm_rbw": 0, "m2l_factored": 0, "pair_order": 4,
            "near_lds": 0, "gemm_lat": 512,
            "gemm_chain": 0, "m2l_cols": 64,
            "gemm_narrow": 0, "near_early": 0, "near_early_grid": 1024, "m2l_early": 0,
            "near_early_start": 0}
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2103_01048_amd", "tuning.json")
SHIPPED_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_table.json")

STAGES = (
    ("work_cap_div", [{"work_cap_div": v} for v in (8192, 16384, 32768, 65536, 131072)]),
    ("tile_split", [{"tile_split2": a, "tile_split4": b} for a, b in ((32, 16), (32, 0), (24, 12), (0, 0))]),
    ("far_weight", [{"far_weight": v} for v in (1.0, 1.15, 1.3)]),
    ("gemm_rbw", [{"gemm_rbw": v} for v in (0, 1, 2, 4)]),
    ("m2l_factored", [{"m2l_factored": v} for v in (0, 1)]),
    ("gemm_narrow", [{"gemm_narrow": v} for v in (0, 1)]),
    # the share of early items and their start together: with pass order 4
    # a split started with the passes is much slower than none, one started
    # after P2M much faster, so one at a time would never take either
    ("near_early", [{"near_early": v, "near_early_start": st} for v in (0, 300, 350, 400, 450, 500, 550)
                    for st in (0, 1) if v or not st]),
    # after the split: the early M2L levels pay off beside the early items
    ("m2l_early", [{"m2l_early": v} for v in (0, 1)]),
    ("pair_order", [{"pair_order": v} for v in (0, 1, 2, 3, 4)]),
    ("near_lds", [{"near_lds": v} for v in (0, 8192, 13312)]),
    ("gemm_lat", [{"gemm_lat": v} for v in (0, 256, 512, 1024)]),
)


def get_tuning() -> dict:
    t = _lib.FmmTuning()
    check(lib().fmm_get_tuning(ctypes.byref(t)), "fmm_get_tuning")
    return {k: getattr(t, k) for k, _ in _lib.FmmTuning._fields_}


def set_tuning(**kw) -> dict:
    """Set tunables for plans set up from now on (unnamed ones keep their
    current values); returns the full set in force."""
    cur = get_tuning()
    unknown = set(kw) - set(cur)
    if unknown:
        raise ValueError(f"unknown tunables {sorted(unknown)}")
    cur.update(kw)
    t = _lib.FmmTuning(**cur)
    check(lib().fmm_set_tuning(ctypes.byref(t)), "fmm_set_tuning")
    return cur


@contextlib.contextmanager
def tuning(**kw):
    """Tunables in force inside the block, restored afterwards."""
    old = get_tuning()
    set_tuning(**kw)
    try:
        yield
    finally:
        set_tuning(**old)


def device_tag(device=None) -> str:
    """The device as the tuning entries name it: its ISA and compute-unit
    count (the marketing name is not reliable on every driver install)."""
    if not torch.cuda.is_available():
        return "cpu"
    pr = torch.cuda.get_device_properties(device)
    arch = (getattr(pr, "gcnArchName", "") or pr.name).split(":")[0]
    return f"{arch}x{pr.multi_processor_count}cu"


def cache_key(n: int, p: int, precision: str, device=None, nmol: int = 1) -> str:
    batch = f"|mol~2^{round(math.log2(nmol))}" if nmol > 1 else ""
    return f"{device_tag(device)}|{precision}|p{p}|n~2^{round(math.log2(max(n, 1)))}{batch}"


def shipped_table() -> dict:
    """Tuning entries that ship with the package (the autotuner's choice for
    the workloads it was run on), consulted after the user's cache."""
    try:
        return json.load(open(SHIPPED_TABLE))
    except (OSError, ValueError):
        return {}


def _time_pair(xt, q, p, ncrit, precision, kappa, steps, warmup, keep, offsets=None, repeats=3):
    pls = [FMMPlan(xt, kernel=k, kappa=kappa, p=p, ncrit=ncrit, precision=precision, offsets=offsets)
           for k in ("laplace", "yukawa")]
    # the latest trial's plans stay alive so that the next trial can share
    # their tree and operators; older ones are released (at millions of
    # points a pair holds gigabytes of pair slots)
    keep[:] = pls
    for _ in range(warmup):
        eval_pair(pls[0], pls[1], q)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(repeats):
        t0 = time.perf_counter()
        for _ in range(steps):
            eval_pair(pls[0], pls[1], q)
        torch.cuda.synchronize()
        best = min(best, (time.perf_counter() - t0) / steps * 1e3)
    return best


def autotune(points: torch.Tensor, p: int = 8, precision: str = "bf16x3", kappa: float = 0.125,
             ncrit_candidates=(64, 96, 128, 160, 192, 256), q: torch.Tensor | None = None, steps: int = 10,
             warmup: int = 10, cache_path: str | None = DEFAULT_CACHE, use_cache: bool = True,
             log=None, offsets=None, repeats: int = 3, width: int = 2) -> dict:
    """Fastest (ncrit, tunables) for pair evaluations on `points` ((N, 3)
    float64 CUDA tensor; with `offsets`, a batch of molecules as FMMPlan
    takes it).  Each trial is the best of `repeats` timings of `steps` pair
    evaluations.  Every ncrit candidate is timed with the defaults;
    the `width` fastest run the stages of coordinate descent each, and the
    fastest of their final settings, timed again side by side, is chosen.
    With use_cache, an entry for this workload in the user's cache
    (cache_path) or else in the package's shipped table is returned without
    a search.  Returns {"key", "ncrit", "tuning", "ms", "trials", "cached"}
    ("source" for a cached entry); the tunables in force are left unchanged
    (see apply)."""
    n = int(points.shape[0])
    nmol = 1 if offsets is None else len(offsets) - 1
    key = cache_key(n, p, precision, points.device, nmol)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        return {**cache[key], "key": key, "cached": True, "source": cache_path}
    shipped = shipped_table() if use_cache else {}
    if key in shipped:
        e = shipped[key]
        return {"ncrit": e["ncrit"], "tuning": {**DEFAULTS, **e["tuning"]}, "ms": e.get("ms"), "key": key,
                "cached": True, "source": "shipped table"}
    xt = points.detach().to(torch.float64).contiguous()
    if q is None:
        g = torch.Generator(device="cpu").manual_seed(0)
        q = torch.randn(n, generator=g, dtype=torch.float64)
    q = q.to(device=xt.device, dtype=torch.float64 if precision == "fp64" else torch.float32)
    trials = []
    old = get_tuning()
    keep = []

    def trial(stage, nc, t):
        set_tuning(**t)
        ms = _time_pair(xt, q, p, nc, precision, kappa, steps, warmup, keep, offsets, repeats)
        trials.append({"stage": stage, "ncrit": nc, "tuning": dict(t), "ms": round(ms, 4)})
        if log:
            log(f"{stage} ncrit {nc} {({k: v for k, v in t.items() if t[k] != DEFAULTS[k]})}: {ms:.4f} ms")
        return ms

    def descend(nc, ms0):
        """The stages one after the other at this ncrit, from the defaults."""
        nonlocal keep
        best_t, best_ms = dict(DEFAULTS), ms0
        for stage, stage_cands in STAGES:
            keep = [pl for pl in keep if pl.ncrit == nc]
            stage_best = (best_ms, None)
            for c in stage_cands:
                t = {**best_t, **c}
                if t == best_t:
                    continue
                ms = trial(stage, nc, t)
                if ms < 0.99 * stage_best[0]:
                    stage_best = (ms, t)
            if stage_best[1] is not None:
                best_ms, best_t = stage_best
        return best_t

    try:
        nc_ms = {nc: trial("ncrit", nc, DEFAULTS) for nc in ncrit_candidates}
        ranked = sorted(nc_ms, key=nc_ms.get)
        # the `width` fastest ncrit values (within 5% of the fastest) each
        # run the stages; their final settings are timed again side by side
        finalists = [nc for nc in ranked[:max(1, width)] if nc_ms[nc] <= 1.05 * nc_ms[ranked[0]]]
        finals = [(nc, descend(nc, nc_ms[nc])) for nc in finalists]
        if len(finals) == 1:
            best_nc, best_t = finals[0]
            best_ms = min(t["ms"] for t in trials if t["ncrit"] == best_nc and t["tuning"] == best_t)
        else:
            timed = [(trial("final", nc, t), nc, t) for nc, t in finals]
            best_ms, best_nc, best_t = min(timed, key=lambda r: r[0])
    finally:
        del keep
        set_tuning(**old)
    res = {"ncrit": best_nc, "tuning": best_t, "ms": round(best_ms, 4), "trials": trials}
    if cache_path:
        cache[key] = {k: res[k] for k in ("ncrit", "tuning", "ms")}
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            tmp = cache_path + ".tmp"
            json.dump(cache, open(tmp, "w"), indent=1)
            os.replace(tmp, cache_path)
        except OSError:
            pass
    return {**res, "key": key, "cached": False}


def apply(result: dict) -> int:
    """Put the tuned parameters in force for plans set up from now on;
    returns the tuned ncrit."""
    set_tuning(**result["tuning"])
    return int(result["ncrit"])
