"""Tuning cache for the plan-specialized matvec.

mrmf_plan_autotune (C ABI) times every candidate shape of the specialized kernel on real buffers and
keeps the fastest in the plan.  This module remembers the winners in a JSON file keyed by the plan's
structure (site dimensions and the operator pattern of every term), the element type and the GPU
architecture, so that later plans with the same structure skip the search.  The cache path is
$MRMF_TUNE_CACHE, else ~/.cache/mrmf/tuning.json; entries measured on MI355X ship with the package in
tuned_gfx950.json and are consulted after the user cache.
"""
from __future__ import annotations

import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SHIPPED = os.path.join(HERE, "tuned_gfx950.json")


def cache_path() -> str:
    return os.environ.get("MRMF_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "mrmf",
                                                              "tuning.json")


def signature(sites, terms, dtype_code: int, arch: str, local_ops=()) -> str:
    """Key of a plan structure: site kinds and dimensions, each term's sites and operators (couplings and
    weights do not change the kernel's shape), the (site, shift) of general one-site operators, the
    element type and the architecture."""
    parts = [arch, str(int(dtype_code))]
    for site, shift in local_ops:
        parts.append(f"l{int(site)}:{int(shift)}")
    for s in sites:
        kind, k = (s.kind, s.k) if hasattr(s, "kind") else s
        parts.append(f"s{int(kind)}:{int(k)}")
    for t in terms:
        if hasattr(t, "site_a"):
            sa, oa, sb, ob = t.site_a, t.op_a, t.site_b, t.op_b
        else:
            sa, oa, sb, ob = t[:4]
        parts.append(f"t{int(sa)},{int(oa)},{int(sb)},{int(ob) if int(sb) >= 0 else 0}")
    return hashlib.sha256("|".join(parts).encode()).hexdigest()[:24]


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(key: str):
    for path in (cache_path(), SHIPPED):
        ent = _load(path).get(key)
        if ent is not None:
            return ent
    return None


def store(key: str, entry: dict, path: str | None = None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    data = _load(path)
    data[key] = entry
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
