"""Autotuner for the performance options of the H/S build.

The tile order changes only the order in which work is dealt to the compute
units, never the arithmetic (bitwise the same H and S); the wave count of the
FP64 contraction also selects its complex form (three real products per
complex one with 8 waves, four with 4), whose results agree to FP64 rounding.
`tune` times the candidates on the caller's inputs with HIP events and
returns the fastest; `cached_options` / `apply` keep the choice in a JSON
cache keyed by device, precision and problem size so later runs reuse it.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, Optional

import torch

from . import _native as N

DEFAULT_CACHE = os.environ.get("HSB_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "hsbuild_tune.json"))
TILE_GROUPS = (0, 4, 8)
WAVES = (4, 8)


def _key(builder, n_g: int, precision: int) -> str:
    prop = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(prop, "gcnArchName", "gpu").split(":")[0]
    k_c = builder.n_atoms * builder.n_l
    # problem-size buckets: the stacked width and the basis size to the next power of two
    return "%s/cu%d/p%d/nl%d/kc%d/ng%d" % (arch, prop.multi_processor_count, precision, builder.n_l,
                                          1 << max(0, (k_c - 1).bit_length()), 1 << max(0, (n_g - 1).bit_length()))


def _load(path: str) -> Dict[str, dict]:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def cached_options(builder, n_g: int, precision: int = N.HSB_FP64, path: str = DEFAULT_CACHE) -> Optional[dict]:
    return _load(path).get(_key(builder, n_g, precision))


def apply(builder, options: dict) -> None:
    if "tile_group" in options:
        builder.set_option(N.HSB_OPT_TILE_GROUP, int(options["tile_group"]))
    if "waves" in options:
        builder.set_option(N.HSB_OPT_HS_WAVES, int(options["waves"]))


def tune(builder, k_frac, g, tau, T, precision: int = N.HSB_FP64, groups: Iterable[int] = TILE_GROUPS,
         waves: Iterable[int] = WAVES, reps: int = 2, path: Optional[str] = DEFAULT_CACHE) -> dict:
    """Times hsbuild_forward for each (waves, tile order) and keeps the fastest
    (and stores it in the cache when `path` is given)."""
    n = int(g.shape[0])
    H = torch.empty((n, n), dtype=torch.complex128, device="cuda")
    S = torch.empty((n, n), dtype=torch.complex128, device="cuda")
    waves = list(waves)
    wsb = 0
    for wv in waves:  # the workspace depends on the wave count (the 8-wave form may split its stacked index)
        builder.set_option(N.HSB_OPT_HS_WAVES, wv)
        wsb = max(wsb, builder.workspace_bytes(N.HSB_MODE_FORWARD, [n]))
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    times = {}
    for wv in waves:
        for gr in groups:
            builder.set_option(N.HSB_OPT_HS_WAVES, wv)
            builder.set_option(N.HSB_OPT_TILE_GROUP, gr)
            code = builder.forward_raw(k_frac, n, g, tau, T, H, S, ws, wsb)  # warm
            if code != N.HSB_OK:
                raise N.HSBuildError(code, N.last_error(builder._h))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                code = builder.forward_raw(k_frac, n, g, tau, T, H, S, ws, wsb)
                if code != N.HSB_OK:
                    raise N.HSBuildError(code, N.last_error(builder._h))
            e1.record()
            torch.cuda.synchronize()
            times[(wv, gr)] = e0.elapsed_time(e1) / reps
    best = min(times, key=times.get)
    builder.set_option(N.HSB_OPT_HS_WAVES, best[0])
    builder.set_option(N.HSB_OPT_TILE_GROUP, best[1])
    result = {"waves": best[0], "tile_group": best[1], "ms": times[best],
              "candidates_ms": {"w%d_g%d" % k: v for k, v in times.items()}}
    if path:
        cache = _load(path)
        cache[_key(builder, n, precision)] = result
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    del H, S, ws
    return result


def tune_batch(builder, k_frac, g_list, tau, T, groups: Iterable[int] = (8, 4), waves: Iterable[int] = (8, 4),
               reps: int = 1) -> dict:
    """Times hsbuild_batch (one captured graph, one persistent contraction over
    every k-point's tiles) for each (waves, tile order) and keeps the fastest.
    Each candidate re-captures the graph once, untimed."""
    times = {}
    H = S = None
    for wv in waves:
        for gr in groups:
            builder.set_option(N.HSB_OPT_HS_WAVES, wv)
            builder.set_option(N.HSB_OPT_TILE_GROUP, gr)
            H, S, _ = builder.batch(k_frac, g_list, tau, T, H, S)  # capture
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                builder.batch(k_frac, g_list, tau, T, H, S)
            e1.record()
            torch.cuda.synchronize()
            times[(wv, gr)] = e0.elapsed_time(e1) / reps
    best = min(times, key=times.get)
    builder.set_option(N.HSB_OPT_HS_WAVES, best[0])
    builder.set_option(N.HSB_OPT_TILE_GROUP, best[1])
    del H, S
    return {"waves": best[0], "tile_group": best[1], "ms": times[best],
            "candidates_ms": {"w%d_g%d" % k: v for k, v in times.items()}}
