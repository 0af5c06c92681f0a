"""Launch settings tuned per shape class.

stba_autotune (in the library) times the Schur assembly for several workgroup
counts and the cluster factorisation in each form that fits, on one problem
and one sample, and writes the fastest into the problem's stba_dims.  This
module keys those choices by a shape class, so that problems of the same
class reuse them without measuring again, and keeps them in a JSON file when
a path is given.
"""
from __future__ import annotations

import json
import math
import os

from . import binding as B

_FORMS = {"auto": B.STBA_CHOL_AUTO, "tiles": B.STBA_CHOL_TILES, "team": B.STBA_CHOL_TEAM,
          "workgroup": B.STBA_CHOL_WORKGROUP}


def shape_class(m: int, q: int, max_track: int, l: int, gamma_max: int, precision: int) -> str:
    """Cameras, observations and clusters to the nearest power of two, the
    padded order of the largest cluster (32-row blocks), whether tracks fit one
    lane group (32 observations), the precision."""
    def p2(x):
        return int(round(math.log2(max(1, x))))
    blocks = (9 * gamma_max + 31) // 32
    return f"m2^{p2(m)}_q2^{p2(q)}_l2^{p2(l)}_T{blocks}_{'short' if max_track <= 32 else 'long'}_p{precision}"


def autotune_solver(solver, sample, cache_path: str | None = None, lam=None, lam_corr: float = 0.1) -> dict:
    """Set solver.dims.chol_form / schur_blocks for `sample`'s shape class: from
    the cache when the class is there, else measured by stba_autotune (and
    stored).  Returns {"class", "chol_form", "schur_blocks", "cached", ...}."""
    key = shape_class(solver.m, solver.q, solver.dims.max_track, sample.l, solver.dims.gamma_max, solver.precision)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
    if key in cache:
        hit = cache[key]
        solver.dims.chol_form = _FORMS[hit["chol_form"]]
        solver.dims.schur_blocks = int(hit["schur_blocks"])
        return {"class": key, "cached": True, **hit}
    lam = lam if lam is not None else solver.read_state()["lambda_"]
    res = B.stba_autotune(solver.problem, solver.dims, sample, B.StbaDamping(lam, lam_corr), solver.precision,
                          solver.ws)
    cache[key] = res
    if cache_path:
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return {"class": key, "cached": False, **res}
