"""Autotuning cache: the fastest kernel variants of a plan shape, measured on
the device by pme_autotune and kept as JSON.

A shape is keyed by (GPU architecture, K1 x K2 x K3, spline order, atom-count
bucket, precision); the bucket is the next power of two of N, so systems of
similar size share an entry.  The cache file is SPME_AUTOTUNE_CACHE, else
~/.cache/paper_2009_12617_amd/autotune.json.  Entries hold the chosen
variants, the measured microseconds per step of every candidate and the
library version that measured them.
"""
import json
import math
import os
import tempfile

import torch

from . import _lib


def cache_path():
    p = os.environ.get("SPME_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2009_12617_amd", "autotune.json")


def n_bucket(n):
    """Next power of two of the atom count (at least 1)."""
    return 1 << max(0, math.ceil(math.log2(max(int(n), 1))))


def arch_name(device):
    props = torch.cuda.get_device_properties(device)
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def shape_key(arch, grid, order, n_atoms, precision):
    K1, K2, K3 = grid
    return f"{arch}/{K1}x{K2}x{K3}/p{order}/n{n_bucket(n_atoms)}/{precision}"


def load(path=None):
    path = path or cache_path()
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def save(entries, path=None):
    """Atomic write (temporary file in the same folder, then rename)."""
    path = path or cache_path()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(os.path.abspath(path)), suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(plan, n_atoms, path=None):
    """The cached variants for this plan's shape and atom count, or None."""
    e = load(path).get(shape_key(arch_name(plan.device), plan.grid, plan.order, n_atoms,
                                 plan.precision))
    if e is None or e.get("version") != _lib.load().pme_version():
        return None
    return e["best"]


def tune(plan, pos, q, box, reps=20, path=None, refresh=False):
    """Set the plan's variants from the cache, measuring them first
    (pme_autotune) when the cache has no entry for this shape or refresh is
    set.  Returns the cache entry."""
    n = int(q.shape[0])
    key = shape_key(arch_name(plan.device), plan.grid, plan.order, n, plan.precision)
    entries = load(path)
    e = entries.get(key)
    if refresh or e is None or e.get("version") != _lib.load().pme_version():
        r = plan.autotune(pos, q, box, reps=reps)
        e = {"best": r["best"], "us_per_step": r["us"], "candidates": r["candidates"],
             "default": plan_default(plan), "version": _lib.load().pme_version(),
             "measured_atoms": n}
        entries = load(path)  # re-read: another process may have added entries
        entries[key] = e
        save(entries, path)
    else:
        plan.set_tuning(**e["best"])
    return e


def plan_default(plan):
    """The built-in variants of the plan's shape."""
    import ctypes
    from .plan import PRECISIONS
    t = _lib.Tuning()
    _lib.check(_lib.load().pme_default_tuning(*plan.grid, plan.order, PRECISIONS[plan.precision],
                                              ctypes.byref(t)), "pme_default_tuning")
    return t.as_dict()
