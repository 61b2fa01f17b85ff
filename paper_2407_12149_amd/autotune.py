"""Autotuner of the sweep kernels: a grid search over the kernel form (LDS
tiles, or register-held stencil with 256 or 512 threads per block) and the
number of chains processed per block, timed on the device through the
library's own update timer, with results cached in a JSON file keyed by
problem shape, precision, chain count and device name."""
import json
import os

from . import mgmc

CANDIDATE_VARIANTS = (1, 2, 0)
CANDIDATE_CPB = (0, 1, 2, 4, 8, 16)


def _key(sampler):
    import torch
    p = sampler.problem
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    return "|".join(str(v) for v in (p["dim"], p["n"], p["levels"], p.get("precision", "fp64"),
                                     sampler.nchains, dev))


def autotune(sampler, cache_path=None, updates=3, verbose=False):
    """Pick the fastest (variant, chains per block) for this sampler, apply it
    and return {"variant": v, "cpb": c, "ms": t, "cached": bool}."""
    key = _key(sampler)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
    if key in cache:
        best = dict(cache[key], cached=True)
    elif sampler.problem["dim"] != 2:
        best = {"variant": 1, "cpb": 0, "ms": None, "cached": False}  # 3D: per-colour kernels
    else:
        results = []
        for v in CANDIDATE_VARIANTS:
            for c in CANDIDATE_CPB:
                if c > sampler.nchains or (v == 0 and c != 0):
                    continue
                sampler.set_option(mgmc.MGMC_OPT_SWEEP_VARIANT, v)
                sampler.set_option(mgmc.MGMC_OPT_CHAINS_PER_BLOCK, c)
                sampler.time_updates(1)  # warm-up
                ms = sampler.time_updates(updates) / updates
                results.append((ms, v, c))
                if verbose:
                    print(f"[autotune] {key} variant={v} cpb={c}: {ms:.3f} ms/update", flush=True)
        ms, v, c = min(results)
        best = {"variant": v, "cpb": c, "ms": ms, "cached": False}
        if cache_path:
            cache[key] = {"variant": v, "cpb": c, "ms": ms}
            tmp = cache_path + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(cache, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache_path)
    sampler.set_option(mgmc.MGMC_OPT_SWEEP_VARIANT, best["variant"])
    sampler.set_option(mgmc.MGMC_OPT_CHAINS_PER_BLOCK, best["cpb"])
    return best
