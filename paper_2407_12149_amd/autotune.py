"""Autotuner of the sweep kernels.

3D contexts tune the chains per thread of their per-site kernels and the
form of the finest sweep (parity passes or one launch per colour).

For every level that runs smoother sweeps (levels >= 1) it searches the
kernel form (LDS tiles, or register-held stencil with 256 or 512 threads per
block, and on the finest, 5-point level also the form whose state tiles come
into LDS by DMA) and the number of chains processed per block, by coordinate descent
from the finest level down: each level's candidates are timed with the
library's own update timer while the other levels keep their current best.
It then tries the bottom levels 0 .. k as one launch for each k.  Results are cached in a JSON
file keyed by problem shape, precision, chain count and device architecture.""" 
import json
import os

from . import mgmc

CANDIDATE_VARIANTS = (1, 2, 0)
FINEST_VARIANTS = (4,)  # LDS DMA state tiles (5-point level only)
MIN_GAIN = 0.005  # a candidate replaces the current choice only when this much faster
CANDIDATE_CPB = (0, 1, 2, 4, 8, 16)


def _key(sampler):
    import torch
    p = sampler.problem
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    dev = f"{getattr(props, 'gcnArchName', '')}:{props.multi_processor_count}"
    return "|".join(str(v) for v in (p["dim"], p["n"], p["levels"], p.get("precision", "fp64"),
                                     sampler.nchains, dev))


def apply(sampler, levels):
    """Set per-level (variant, chains per block) pairs; None entries reset."""
    for l, vc in enumerate(levels):
        v, c = (-1, -1) if vc is None else vc
        sampler.set_level_option(l, mgmc.MGMC_OPT_SWEEP_VARIANT, v)
        sampler.set_level_option(l, mgmc.MGMC_OPT_CHAINS_PER_BLOCK, c)


def _time(sampler, updates):
    """Milliseconds per update: the best of three runs of `updates` updates."""
    sampler.time_updates(2)  # warm-up
    return min(sampler.time_updates(updates) / updates for _ in range(3))


def autotune(sampler, cache_path=None, updates=8, verbose=False):
    """Pick the fastest per-level settings for this sampler, apply them and
    return {"levels": [[variant, cpb] or None per level], "ms": t, "cached": bool}."""
    key = _key(sampler)
    nlev = int(sampler.problem["levels"])
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
    if key in cache and "levels" in cache[key]:
        best = dict(cache[key], cached=True)
    elif sampler.problem["dim"] == 3:
        best = dict(_tune_3d(sampler, updates, verbose, key), cached=False)
        if cache_path:
            cache[key] = {k: v for k, v in best.items() if k != "cached"}
            tmp = cache_path + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(cache, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache_path)
    elif nlev < 2:
        best = {"levels": [None] * nlev, "ms": None, "cached": False}  # per-colour kernels
    else:
        sampler.set_option(mgmc.MGMC_OPT_SWEEP_VARIANT, 3)
        sampler.set_option(mgmc.MGMC_OPT_CHAINS_PER_BLOCK, 0)
        levels = [None] * nlev
        apply(sampler, levels)
        ms_best = _time(sampler, updates)
        for l in range(nlev - 1, 0, -1):
            choice = None
            for v in CANDIDATE_VARIANTS + (FINEST_VARIANTS if l == nlev - 1 else ()):
                for c in CANDIDATE_CPB:
                    if c > sampler.nchains or (v == 0 and c != 0):
                        continue
                    sampler.set_level_option(l, mgmc.MGMC_OPT_SWEEP_VARIANT, v)
                    sampler.set_level_option(l, mgmc.MGMC_OPT_CHAINS_PER_BLOCK, c)
                    ms = _time(sampler, updates)
                    if verbose:
                        print(f"[autotune] {key} level {l} variant={v} cpb={c}: {ms:.3f} ms/update",
                              flush=True)
                    if ms < ms_best * (1.0 - MIN_GAIN):
                        ms_best, choice = ms, [v, c]
            if choice is not None:
                levels[l] = choice
            apply(sampler, levels)
        # the bottom levels 0 .. k as one launch, if that is faster (the
        # library caps k at the deepest level it can fuse)
        fused = 0
        for k in range(1, min(nlev - 1, 6)):
            sampler.set_option(mgmc.MGMC_OPT_COARSE_FUSED, k)
            ms = _time(sampler, updates)
            if verbose:
                print(f"[autotune] {key} fused bottom 0..{k}: {ms:.3f} ms/update", flush=True)
            if ms < ms_best * (1.0 - MIN_GAIN):
                ms_best, fused = ms, k
        sampler.set_option(mgmc.MGMC_OPT_COARSE_FUSED, fused)
        best = {"levels": levels, "fused": fused, "ms": ms_best, "cached": False}
        if cache_path:
            cache[key] = {"levels": levels, "fused": fused, "ms": ms_best}
            tmp = cache_path + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(cache, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache_path)
    if sampler.problem["dim"] == 3:
        sampler.set_option(mgmc.MGMC_OPT_TILED_SWEEPS, int(best.get("parity", 1)))
        sampler.set_option(mgmc.MGMC_OPT_CHAINS_PER_BLOCK, int(best.get("cpb", 0)))
        return best
    sampler.set_option(mgmc.MGMC_OPT_SWEEP_VARIANT, 3)
    sampler.set_option(mgmc.MGMC_OPT_CHAINS_PER_BLOCK, 0)
    sampler.set_option(mgmc.MGMC_OPT_COARSE_FUSED, int(best.get("fused", 0)))
    apply(sampler, best["levels"])
    return best


def _tune_3d(sampler, updates, verbose, key):
    """3D contexts: the chains per thread of the per-site kernels (by size,
    or forced to 1 .. 16) and, on the 7-point finest level, parity passes or
    one launch per colour; coordinate descent, forced groups first."""
    nlev = int(sampler.problem["levels"])
    choice = {"parity": 1, "cpb": 0}
    sampler.set_option(mgmc.MGMC_OPT_TILED_SWEEPS, 1)
    sampler.set_option(mgmc.MGMC_OPT_CHAINS_PER_BLOCK, 0)
    ms_best = _time(sampler, updates)
    for c in (1, 2, 4, 8, 16):
        if c > sampler.nchains:
            continue
        sampler.set_option(mgmc.MGMC_OPT_CHAINS_PER_BLOCK, c)
        ms = _time(sampler, updates)
        if verbose:
            print(f"[autotune] {key} 3D chains per thread {c}: {ms:.3f} ms/update", flush=True)
        if ms < ms_best * (1.0 - MIN_GAIN):
            ms_best, choice["cpb"] = ms, c
    sampler.set_option(mgmc.MGMC_OPT_CHAINS_PER_BLOCK, choice["cpb"])
    sampler.set_option(mgmc.MGMC_OPT_TILED_SWEEPS, 0)
    ms = _time(sampler, updates)
    if ms < ms_best * (1.0 - MIN_GAIN):
        ms_best, choice["parity"] = ms, 0
    sampler.set_option(mgmc.MGMC_OPT_TILED_SWEEPS, choice["parity"])
    return {"levels": [None] * nlev, "ms": ms_best, **choice}
