"""Autotuner of the MD step's launch configuration.

Four knobs change only the speed of a run, never its physics:

* the step form: "walk" (one pass; partner sums by walking the partner's
  list) or "sums" (two passes through per-particle switching sums), the
  same energy written two ways (results differ by rounding order),
* the gather width of the fused step kernel (flattened list entries each
  lane evaluates per pass: 1, 2 or 4; every width gives the same bits),
* the steps per replayed graph (graph_steps),
* the neighbour-list skin r_buff (longer lists against fewer rebuilds; the
  trajectory changes only by rounding order).

``autotune`` times short runs of every candidate, each on a fresh copy of the
workload (``factory(r_buff)`` builds a new ``System`` or ``Batch`` from the
same start, so every candidate runs the same stretch of the trajectory: a
relaxing start rebuilds its lists more often than a settled one) and returns
the fastest; results are cached in a JSON file keyed by a workload signature,
so a second call with the same signature costs nothing.
"""
from __future__ import annotations

import itertools
import json
import os
import time
from typing import Callable, Dict, Optional, Sequence

import torch

DEFAULT_CACHE = os.environ.get("RC_TUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                              "_tune_cache.json"))


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(factory: Callable[[float], object], cfg, signature: str, r_buffs: Sequence[float],
             widths: Sequence[int] = (1, 2, 4), graph_steps: Sequence[int] = (16, 32),
             forms: Sequence[str] = ("walk", "sums"), steps: int = 200, warmup: int = 60,
             cache: Optional[str] = DEFAULT_CACHE, log=None) -> Dict:
    """Fastest (r_buff, form, width, graph_steps) for the workload built by factory.

    Every candidate runs ``steps`` steps (after ``warmup`` untimed ones per
    r_buff) with the graph-replaying driver; the time per step includes the
    rebuilds and the chunk bookkeeping the driver does.
    """
    if cache:
        hit = _load(cache).get(signature)
        if hit:
            return hit
    results = []
    for rb in r_buffs:
        for form, w, G in itertools.product(forms, widths, graph_steps):
            obj = factory(float(rb))
            obj.set_step_form(form)
            obj.set_gather_width(int(w))
            obj.run(warmup, cfg, step0=0, graph_steps=int(G))   # graphs built, caches warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = obj.run(steps, cfg, step0=warmup, graph_steps=int(G))
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            results.append({"r_buff": float(rb), "form": form, "width": int(w), "graph_steps": int(G),
                            "us_per_step": dt / steps * 1e6, "rebuilds": int(r.stats.rebuilds)})
            if log:
                log(f"tune {signature}: r_buff {rb} {form} width {w} graph_steps {G}: "
                    f"{dt / steps * 1e6:.2f} us/step, {int(r.stats.rebuilds)} builds")
            del obj
        torch.cuda.empty_cache()
    best = min(results, key=lambda x: x["us_per_step"])
    out = dict(best)
    out["candidates"] = results
    if cache:
        data = _load(cache)
        data[signature] = out
        _store(cache, data)
    return out
