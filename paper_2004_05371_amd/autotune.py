"""Plan cache of the autotuner.

The search itself runs in the library (``red_autotune`` /
``red_autotune_segmented``: the nontemporal hint, workgroup size x loads
per thread, grid size and synchronization variant, timed with HIP events
on the caller's data; the segmented search re-times its best candidates in
interleaved rounds).  This module persists its
results as JSON and installs them into the library's plan table:

    {"format": 1, "arch": "gfx950", "cus": 256,
     "entries": [{"kind": "sum", "dtype": "f32", "acc": "compensated",
                  "n": 268435456, "plan": {...}, "us": 150.2}, ...]}

Plans are keyed in the library by (dtype, accumulation, ceil(log2 n)) for
sums and by ceil(log2 nseg) for segmented batches.  A missing, corrupt or
foreign cache installs nothing and leaves the default plans in place.
"""
from __future__ import annotations

import json
import os
import warnings
from typing import List, Optional

from . import redsum as R

PKG = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(PKG, "tuned_plans.json")
CACHE_ENV = "REDSUM_TUNE_CACHE"
FORMAT = 1

DTYPES = {"i32": R.RED_I32, "f32": R.RED_F32, "f16": R.RED_F16, "bf16": R.RED_BF16}
ACCS = {"compensated": R.RED_ACC_COMPENSATED, "plain": R.RED_ACC_PLAIN}
VARIANTS = {"relaunch": R.RED_VARIANT_RELAUNCH, "atomic": R.RED_VARIANT_ATOMIC,
            "persistent": R.RED_VARIANT_PERSISTENT, "single": R.RED_VARIANT_SINGLE}


def cache_path(path: Optional[str] = None) -> str:
    return path or os.environ.get(CACHE_ENV) or DEFAULT_CACHE


def plan_from_dict(d: dict) -> R.Plan:
    v = d["variant"]
    v = VARIANTS[v] if isinstance(v, str) else int(v)
    return R.Plan(v, int(d["wg"]), int(d["ipt"]), int(d["grid"]), int(d.get("flags", 0)))


def load(path: Optional[str] = None, arch: str = "gfx950") -> int:
    """Install every valid plan of the cache; returns how many.  Problems
    are reported as warnings, never raised."""
    p = cache_path(path)
    try:
        with open(p) as fh:
            doc = json.load(fh)
    except FileNotFoundError:
        return 0
    except (OSError, ValueError) as e:
        warnings.warn("plan cache %s unreadable (%s); using default plans" % (p, e))
        return 0
    if not isinstance(doc, dict) or doc.get("format") != FORMAT or doc.get("arch") != arch:
        warnings.warn("plan cache %s has another format or architecture; using default plans" % p)
        return 0
    n = 0
    for e in doc.get("entries", []):
        try:
            plan = plan_from_dict(e["plan"])
            if e["kind"] == "sum":
                rc = R.load().red_set_plan(DTYPES[e["dtype"]], ACCS[e["acc"]], int(e["n"]), plan)
            elif e["kind"] == "segmented":
                rc = R.load().red_set_segmented_plan(int(e["nseg"]), plan)
            else:
                continue
        except (KeyError, TypeError, ValueError) as ex:
            warnings.warn("plan cache entry skipped: %r (%s)" % (e, ex))
            continue
        if rc == R.RED_OK:
            n += 1
        else:
            warnings.warn("plan cache entry rejected by the library: %r (%s)" % (e, R.last_error()))
    return n


def bucket(n: int) -> int:
    """ceil(log2 n): the library's plan-table bucket of an element count."""
    return max(0, (int(n) - 1).bit_length())


def entry_key(e: dict):
    if e.get("kind") == "sum":
        return ("sum", e["dtype"], e["acc"], bucket(e["n"]))
    return ("segmented", bucket(e["nseg"]))


def cached_keys(path: Optional[str] = None) -> set:
    """Keys of the entries of a readable cache (no validation)."""
    try:
        with open(cache_path(path)) as fh:
            doc = json.load(fh)
        return {entry_key(e) for e in doc.get("entries", [])}
    except (OSError, ValueError, KeyError, TypeError, AttributeError):
        return set()


def save(entries: List[dict], path: Optional[str] = None, cus: int = 256, arch: str = "gfx950") -> str:
    p = cache_path(path)
    doc = {"format": FORMAT, "arch": arch, "cus": cus, "entries": entries}
    tmp = p + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(doc, fh, indent=1)
    os.replace(tmp, p)
    return p


def tune_sum(t, out, acc: int = R.RED_ACC_COMPENSATED, stream: Optional[int] = None, budget: int = 0) -> dict:
    """Autotune red_sum for tensor `t` (overwrites `out`) and return the
    cache entry of the installed plan."""
    code = R.dtype_code(t)
    s = R.current_stream() if stream is None else stream
    plan, us = R.red_autotune(code, acc, t.data_ptr(), t.numel(), out.data_ptr(), s, budget)
    inv_d = {v: k for k, v in DTYPES.items()}
    inv_a = {v: k for k, v in ACCS.items()}
    return {"kind": "sum", "dtype": inv_d[code], "acc": inv_a[acc], "n": int(t.numel()),
            "plan": plan.as_dict(), "us": round(us, 2)}


def tune_segmented(values, offsets, out, stream: Optional[int] = None, budget: int = 0) -> dict:
    s = R.current_stream() if stream is None else stream
    nseg = offsets.numel() - 1
    plan, us = R.red_autotune_segmented(values.data_ptr(), offsets.data_ptr(), nseg, out.data_ptr(), s, budget)
    return {"kind": "segmented", "nseg": int(nseg), "total": int(values.numel()), "plan": plan.as_dict(),
            "us": round(us, 2)}
