"""Autotuner results kept across runs.

ttsh_tune times the candidate launch configurations of the two step passes
(workgroup size, one launch for all grid sizes or one per size, transform
schedule, one or two concurrent instance groups) and keeps the fastest; the
choice depends only on the mix of grid sizes, the arithmetic, whether the
vorticity-damping term is on, and the device.  This module keeps a JSON file
of choices under that key, so that a later run sets the configuration
(ttsh_set_tuning) without timing anything.

The file maps key -> {"cfg": [7 ints, as ttsh_tune], "us_per_step": float
(whole steps)}; a cfg of 6 ints (without the group count) means one group.
A missing or unreadable file reads as empty; writes replace the file
atomically.
"""
from __future__ import annotations

import json
import os
from collections import Counter
from pathlib import Path

from . import ttsh as T

DEFAULT_CACHE = Path(__file__).resolve().with_name("tuning_cache.json")


def cache_key(Ns, precision: int, gw: bool, arch: str) -> str:
    """'arch|p<precision>|gw<0/1>|<count>x<N>,...' with the grid sizes in
    increasing order; the order of the instances does not matter."""
    mix = ",".join(f"{n}x{N}" for N, n in sorted(Counter(int(v) for v in Ns).items()))
    return f"{arch}|p{int(precision)}|gw{int(bool(gw))}|{mix}"


def load(path=DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return {}
    return d if isinstance(d, dict) else {}


def store(key: str, cfg, us: float, path=DEFAULT_CACHE) -> None:
    d = load(path)
    d[key] = {"cfg": [int(v) for v in cfg], "us_per_step": float(us)}
    path = Path(path)
    tmp = path.with_name(path.name + ".tmp")
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(solver, nsteps: int = 20, path=DEFAULT_CACHE, retune: bool = False, write: bool = True):
    """Apply the cached configuration for the solver's context if there is
    one (and retune is False), else run the tuner and record its choice
    (write=False keeps the file untouched).  Returns (cfg, us_per_step or
    None, hit)."""
    key = cache_key(solver.N, solver.precision, solver.gw, T.ttsh_device_arch())
    entry = None if retune else load(path).get(key)
    if entry is not None:
        try:
            solver.set_tuning(entry["cfg"])
            return tuple(entry["cfg"]), entry.get("us_per_step"), True
        except (T.TTSHError, KeyError, TypeError, ValueError):
            pass  # a stale or malformed entry: tune again
    cfg, us = solver.tune(nsteps)
    if write:
        try:
            store(key, cfg, us, path)
        except OSError:
            pass  # a read-only tree: the choice still applies to this run
    return cfg, us, False
