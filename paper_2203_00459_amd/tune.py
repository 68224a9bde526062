"""Autotuning of the search's launch choices, with a JSON cache.

The library's fmbym_autotune times whole search steps for each column pass at
4, 8 and 16 columns per block, the batch split, the rows per line of the row
passes and the radix plan of the n-point column lines, and keeps the fastest
(only the radix plans change results, by FP32 rounding).  This module keys
the outcome by (GPU architecture, n, n_theta, n_r, batch, pass) and stores it
in a JSON file, so a later process sets the choices without measuring again;
an entry without every current field is measured again.
"""
from __future__ import annotations

import json
import os

import torch

from . import fmbym


def default_cache_path() -> str:
    return os.environ.get("FMBYM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "fmbym", "tuning.json"))


def cache_key(search: "fmbym.Search", batch: int, with_backward: bool) -> str:
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    p = search.params
    return f"{arch}/n{p.n}/t{p.n_theta}/r{p.n_r}/b{batch}/{'fwd+bwd' if with_backward else 'fwd'}"


def _load(path: str) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def autotune(search: "fmbym.Search", batch: int, with_backward: bool = True, cache_path: str | None = None,
             refresh: bool = False) -> dict:
    """Set the plan's widths from the cache, or measure and store them.
    Returns {"tuning": {...}, "ms_per_step": float | None, "from_cache": bool}."""
    path = cache_path or default_cache_path()
    key = cache_key(search, batch, with_backward)
    cache = _load(path)
    if not refresh and key in cache and set(fmbym.TUNING_FIELDS) <= set(cache[key].get("tuning", {})):
        fmbym.plan_set_tuning(search.plan, cache[key]["tuning"])
        return dict(cache[key], from_cache=True)
    tuning, ms = fmbym.plan_autotune(search.plan, batch, with_backward, torch.device("cuda"))
    cache = _load(path)
    cache[key] = {"tuning": tuning, "ms_per_step": ms}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return {"tuning": tuning, "ms_per_step": ms, "from_cache": False}
