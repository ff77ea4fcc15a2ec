"""Autotuner driver: runs the library's successive-halving search
(rx_autotune / rx_autotune_multi) and caches the winning launch shape as JSON,
keyed by device architecture, workload kind, program size class and string
length class.  A cached entry is reused without re-timing."""
from __future__ import annotations

import ctypes
import json
import math
import os

from . import rx

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "rx_mi355x_tune.json")


def _cls(x: float) -> int:
    return int(math.ceil(math.log2(max(1.0, float(x)))))


def _arch() -> str:
    import torch

    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, cache):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def key_single(prog: rx.Program, n: int, mean_len: float, fixed: bool) -> str:
    jit = prog.jit_stats()["ready"] if fixed else 0
    return f"{_arch()}|single|{'fixed' if fixed else 'offsets'}|jit{jit}|L{_cls(prog.info.n_leaves)}|" \
           f"W{prog.info.words}|len{_cls(mean_len)}|n{_cls(n)}"


def tune_single(prog: rx.Program, data, offsets=None, length=0, n=None, budget_runs=64, cache_path=None,
                use_cache=True):
    """Best rx_launch for rx_match (offsets given) or rx_match_fixed (length given).
    Returns (launch, info dict)."""
    import torch

    cache_path = cache_path or DEFAULT_CACHE
    fixed = offsets is None
    if n is None:
        n = (data.numel() // length) if fixed else offsets.numel() - 1
    mean_len = length if fixed else float((offsets[-1] - offsets[0]).item()) / max(n, 1)
    key = key_single(prog, n, mean_len, fixed)
    cache = _load(cache_path) if use_cache else {}
    if key in cache:
        c = cache[key]
        return rx.rx_launch(c["variant"], c["block"], c["grid"], c.get("unroll", 0)), dict(c, cached=True)
    if prog._dev_buf is None:
        prog.upload(device=data.device)
    out = torch.empty(n, dtype=torch.uint8, device=data.device)
    best = rx.rx_launch()
    ms = ctypes.c_double()
    nc = ctypes.c_int32()
    rx._check(rx.lib().rx_autotune(prog.handle, ctypes.c_void_p(data.data_ptr()),
                                   None if fixed else ctypes.c_void_p(offsets.data_ptr()), int(length), int(n),
                                   ctypes.c_void_p(out.data_ptr()), int(budget_runs), ctypes.byref(best),
                                   ctypes.byref(ms), ctypes.byref(nc), rx._stream_handle()))
    rec = {"variant": best.variant, "block": best.block, "grid": best.grid, "unroll": best.unroll,
           "ms": ms.value, "candidates": nc.value}
    cache[key] = rec
    _store(cache_path, cache)
    return best, dict(rec, cached=False)


def tune_multi(progs, data, offsets, budget_runs=96, cache_path=None, use_cache=True, planes=False):
    """Best rx_multi_config for rx_match_multi.  Returns (config, info dict).  planes: also try the
    plane form (the list must be prepared with rx.prepare_multi)."""
    import torch

    cache_path = cache_path or DEFAULT_CACHE
    n = offsets.numel() - 1
    mean_len = float((offsets[-1] - offsets[0]).item()) / max(n, 1)
    lmax = max(p.info.n_leaves for p in progs)
    key = f"{_arch()}|multi|P{len(progs)}|L{_cls(lmax)}|len{_cls(mean_len)}|n{_cls(n)}|planes{int(planes)}"
    cache = _load(cache_path) if use_cache else {}
    if key in cache:
        c = cache[key]
        return rx.multi_config(c["edges"], c["block"], c["grid"], c.get("form", 0), c.get("max_bytes", 0)), \
            dict(c, cached=True)
    for p in progs:
        if p._dev_buf is None:
            p.upload(device=offsets.device)
    worst = rx.multi_config(list(range(1, 16)), 64, 0)
    need = rx.lib().rx_match_multi_workspace(n, len(progs), ctypes.byref(worst))
    if need < 0:
        rx._check(int(need))
    if planes:
        # room for the plane form too (the tuner tries it when the list has its module)
        pc = rx.multi_config(form=rx.FORM_PLANES, max_bytes=int((offsets[-1] - offsets[0]).item()))
        need = max(need, rx.lib().rx_match_multi_workspace(n, len(progs), ctypes.byref(pc)))
    work = torch.empty(int(need) + 256, dtype=torch.uint8, device=offsets.device)
    wptr = work.data_ptr() + ((-work.data_ptr()) % 256)
    out = torch.empty((len(progs), n), dtype=torch.uint8, device=offsets.device)
    handles = (ctypes.c_void_p * len(progs))(*[p.handle.value for p in progs])
    best = rx.rx_multi_config()
    ms = ctypes.c_double()
    nc = ctypes.c_int32()
    rx._check(rx.lib().rx_autotune_multi(handles, len(progs), ctypes.c_void_p(data.data_ptr()),
                                         ctypes.c_void_p(offsets.data_ptr()), n, ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(wptr), int(need), int(budget_runs), ctypes.byref(best),
                                         ctypes.byref(ms), ctypes.byref(nc), rx._stream_handle()))
    rec = {"edges": [best.edges[i] for i in range(best.n_edges)], "block": best.block, "grid": best.grid,
           "form": best.form, "max_bytes": best.max_bytes, "ms": ms.value, "candidates": nc.value}
    cache[key] = rec
    _store(cache_path, cache)
    return best, dict(rec, cached=False)
