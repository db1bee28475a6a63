"""Launch-shape autotuner for the registration kernels.

The library exposes process-wide launch-shape tunables (sweep blocks, the
forward sweep's plane-marching tiles, the backward sweep's staged threshold,
the x-pass LDS budget, the y / z tile columns); none of them changes a result
beyond the order of the FP64 energy sums, only the speed.  `autotune` times a short fixed-step registration of the caller's own
problems (their pyramid, a few iterations per level) for each candidate value, one tunable at a time (coordinate search from
the defaults), keeps the fastest, and caches the choice in a JSON file keyed by
architecture, T and the computational grids.  `apply` sets a cached choice.
"""

from __future__ import annotations

import json
import os
import time

import torch

from . import lddmm as L

DEFAULTS = {L.TUNE_SWEEP_BLOCKS: 4096, L.TUNE_FWD_TILES: 1792, L.TUNE_STAGED_MIN_BLOCKS: 2048,
            L.TUNE_FFT_X_ELEMS: 2048, L.TUNE_FFT_COLS: 16, L.TUNE_FFT_ZCOLS: 8,
            L.TUNE_FWD_STAGED_MIN_BLOCKS: 2048}
CANDIDATES = {
    L.TUNE_SWEEP_BLOCKS: (512, 1024, 2048, 4096),
    L.TUNE_FWD_TILES: (0, 1792, 2048, 3584, 4096),
    L.TUNE_STAGED_MIN_BLOCKS: (1, 1024, 2048, 1 << 30),
    L.TUNE_FFT_X_ELEMS: (1024, 2048, 4096),
    L.TUNE_FFT_COLS: (4, 8, 16, 32),
    L.TUNE_FFT_ZCOLS: (4, 8, 16, 32),
    L.TUNE_FWD_STAGED_MIN_BLOCKS: (1, 1024, 2048, 1 << 30),
}
NAMES = {L.TUNE_SWEEP_BLOCKS: "sweep_blocks", L.TUNE_FWD_TILES: "fwd_tiles",
         L.TUNE_STAGED_MIN_BLOCKS: "staged_min_blocks",
         L.TUNE_FFT_X_ELEMS: "fft_x_elems",
         L.TUNE_FFT_COLS: "fft_cols", L.TUNE_FFT_ZCOLS: "fft_zcols",
         L.TUNE_FWD_STAGED_MIN_BLOCKS: "fwd_staged_min_blocks"}


def cache_path():
    return os.environ.get("LDDMM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "lddmm_tune.json"))


def arch():
    if not torch.cuda.is_available():
        return "none"
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def key(shapes, params: L.Params, spacing=1.0):
    """Cache key: architecture, T and the finest computational grid of each problem."""
    grids = [L.lddmm_comp_grid(tuple(s), params, params.n_levels - 1, spacing) for s in shapes]
    return f"{arch()}|T{params.T}|" + ";".join("x".join(str(n) for n in g) for g in grids)


def _load_cache():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(cache):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass                      # read-only home: the choice stays in memory only


def set_all(choice):
    for which, value in choice.items():
        L.lddmm_set_tunable(int(which), int(value))


def _run_once(pairs, params, wss):
    if len(pairs) == 1:
        d = pairs[0]
        L.lddmm_register(d["M0"], d["M1"], d.get("MI0"), d.get("MI1"), params=params,
                         spacing=d.get("spacing", 1.0), ws=wss[0], want_phi=False)
    else:
        L.lddmm_register_batched(pairs, params, wss=wss, want_phi=False)


# A candidate replaces the current value only when it is at least this much
# faster: trial times of a few iterations vary by about 1 % from run to run, and
# the plain minimum then picked shapes that were slower over a whole registration.
MARGIN = 0.01


def autotune(pairs, params: L.Params, iters=3, repeats=3, use_cache=True, verbose=False):
    """Pick the fastest launch shapes for these problems (list of dicts with M0, M1,
    optional MI0, MI1, spacing).  Returns {tunable id: value}; leaves them set."""
    shapes = [tuple(d["M0"].shape) for d in pairs]
    spacing = pairs[0].get("spacing", 1.0)
    k = key(shapes, params, spacing)
    cache = _load_cache() if use_cache else {}
    if k in cache:
        choice = {int(w): v for w, v in cache[k].items()}
        set_all(choice)
        return choice
    # the caller's pyramid with a few iterations per level: a launch shape can
    # help the finest grid and hurt the coarse ones (the staged-sweep threshold)
    short = L.Params(alpha=params.alpha, gamma=params.gamma, sigma=params.sigma, T=params.T,
                     n_levels=params.n_levels, iters=(iters,) * params.n_levels,
                     step=params.step, guard=False, weight=params.weight, flags=params.flags)
    wss = [L.workspace(s, short, d.get("spacing", 1.0), d["M0"].device)
           for s, d in zip(shapes, pairs)]
    choice = dict(DEFAULTS)
    set_all(choice)
    _run_once(pairs, short, wss)                      # warm up code objects and tables
    torch.cuda.synchronize()

    def timed():
        best = float("inf")
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _run_once(pairs, short, wss)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best

    for which, values in CANDIDATES.items():
        current = choice[which]
        times = {}
        for v in (current,) + tuple(x for x in values if x != current):
            choice[which] = v
            set_all(choice)
            times[v] = timed()
        best = min(times, key=times.get)
        choice[which] = best if times[best] < (1.0 - MARGIN) * times[current] else current
        if verbose:
            print(NAMES[which], {v: round(t * 1e3, 3) for v, t in times.items()}, "->",
                  choice[which])
    set_all(choice)
    if use_cache:
        cache = _load_cache()
        cache[k] = {str(w): v for w, v in choice.items()}
        _store_cache(cache)
    return choice


def apply(shapes, params: L.Params, spacing=1.0):
    """Set the cached choice for these grids if there is one; else the defaults.
    Returns the values set."""
    c = _load_cache().get(key(shapes, params, spacing))
    choice = {int(w): v for w, v in c.items()} if c else dict(DEFAULTS)
    set_all(choice)
    return choice
