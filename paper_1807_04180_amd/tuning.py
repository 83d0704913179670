"""Autotuner of the block substitution with a persistent plan cache.

The search space is the factor layout (two-ended or one-directional
elimination), the substitution variant (one launch per block, one
workgroup per chain, split chains, matrix-core tiles) and, for the chain
variant on batches of more than 4 right-hand sides, its RHS tile (4, 8 or
16; the tile fixes the workgroup size, see include/ddm.h).  Every candidate
the handle admits is timed on the handle's own shapes through the C-ABI
(ddm_time_local_solve); the fastest is applied and stored in a JSON file
keyed by (GPU architecture, dimension, largest block, blocks per chain,
subdomains, RHS count, precision), so that another handle of the same shape
takes the plan without timing.  Everything here is host-side bookkeeping;
the timing runs in libddm.
"""
from __future__ import annotations

import json
import os
import threading
from typing import Dict, List, Optional, Tuple

import torch

from .solver import DDMError, HelmholtzDDM

DEFAULT_PATH = os.environ.get(
    "DDM_TUNING_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "paper_1807_04180_amd", "tuning.json"))

VARIANTS = ("perline", "chain", "chain2", "mma")


def _shape(s: HelmholtzDDM) -> Tuple[int, int]:
    """(largest block size, most blocks per subdomain) from the boxes."""
    bs_max = nb_max = 0
    for a in range(s.nsub):
        g = s.geometry(a)
        ext = [g["ext_hi"][d] - g["ext_lo"][d] + 1 for d in range(s.problem.dim)]
        nb = ext[-1]
        bs = 1
        for e in ext[:-1]:
            bs *= e
        bs_max, nb_max = max(bs_max, bs), max(nb_max, nb)
    return bs_max, nb_max


def plan_key(s: HelmholtzDDM, nrhs: int, scope: str = "") -> str:
    """Cache key of a shape; scope names a restricted search (e.g. "onedir")."""
    props = torch.cuda.get_device_properties(s.device)
    arch = getattr(props, "gcnArchName", None) or props.name
    bs_max, nb_max = _shape(s)
    parts = [str(arch).split(":")[0], "dim%d" % s.problem.dim, "bs%d" % bs_max, "nb%d" % nb_max,
             "nsub%d" % s.nsub, "nrhs%d" % nrhs, "mixed" if s.problem.mixed else "fp64"]
    if scope:
        parts.append(scope)
    return "|".join(parts)


class PlanCache:
    """JSON file of tuned plans; safe to share between threads of one process."""

    def __init__(self, path: str = DEFAULT_PATH):
        self.path = path
        self._lock = threading.Lock()
        self._plans: Dict[str, dict] = {}
        if os.path.exists(path):
            try:
                with open(path) as fh:
                    self._plans = json.load(fh)
            except (OSError, ValueError):
                self._plans = {}

    def get(self, key: str) -> Optional[dict]:
        with self._lock:
            p = self._plans.get(key)
            return dict(p) if p else None

    def put(self, key: str, plan: dict):
        with self._lock:
            self._plans[key] = dict(plan)
            d = os.path.dirname(self.path)
            if d:
                os.makedirs(d, exist_ok=True)
            tmp = "%s.tmp%d" % (self.path, os.getpid())
            with open(tmp, "w") as fh:
                json.dump(self._plans, fh, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def scope_of(layouts: Tuple[bool, ...]) -> str:
    """Cache scope of a layout restriction ("" for the full search)."""
    t = tuple(sorted(set(bool(x) for x in layouts)))
    return {(False, True): "", (False,): "onedir", (True,): "twisted"}[t]


def apply_plan(s: HelmholtzDDM, plan: dict):
    """Put the handle in the plan's configuration and factorise it once in
    that configuration (the layout and the order of the stored inverses
    follow the plan)."""
    s.set_factor_layout(bool(plan["twisted"]), refactor=False)
    s.set_solve_variant(plan["variant"])  # unfactored now: nothing is re-run here
    s.set_chain_tile(int(plan.get("chain_tile", 0)))
    s.factor()


def tune(s: HelmholtzDDM, nrhs: Optional[int] = None, reps: int = 3, cache: Optional[PlanCache] = None,
         force: bool = False, layouts: Tuple[bool, ...] = (True, False)) -> dict:
    """Time every admissible (layout, variant, tile) on this handle, apply the
    fastest and record it.  With a cache hit (and not force) the cached plan
    is applied without timing.  layouts restricts the factor layouts tried
    (True = two-ended, False = one-directional): the two-ended substitution
    waits between the two chains of a subdomain and is launched
    cooperatively, and a cooperative launch does not run beside kernels of
    other streams, so a caller that runs many handles at once may want
    (False,) only.  Returns the plan: twisted, variant, chain_tile, ms (its
    time per local solve) and the table of all timings."""
    nrhs = int(nrhs or s.nrhs_max)
    layouts = tuple(bool(t) for t in layouts)
    key = plan_key(s, nrhs, scope_of(layouts))
    if cache is not None and not force:
        plan = cache.get(key)
        if plan is not None:
            apply_plan(s, plan)
            plan["cached"] = True
            return plan
    table: List[dict] = []
    for twisted in layouts:
        try:
            s.set_factor_layout(twisted)
        except DDMError:
            continue
        for v in VARIANTS:
            try:
                s.set_solve_variant(v)
            except DDMError:
                continue
            tiles = (4, 8, 16) if (v == "chain" and nrhs > 4) else (0,)
            for t in tiles:
                s.set_chain_tile(t)
                try:
                    ms = s.time_local_solve(nrhs, reps)
                except DDMError:
                    continue
                table.append({"twisted": twisted, "variant": v, "chain_tile": t, "ms": ms})
            s.set_chain_tile(0)
    if not table:
        raise RuntimeError("no substitution configuration could be timed")
    best = min(table, key=lambda r: r["ms"])
    plan = {"twisted": best["twisted"], "variant": best["variant"], "chain_tile": best["chain_tile"],
            "ms": best["ms"], "table": table, "key": key}
    apply_plan(s, plan)
    if cache is not None:
        cache.put(key, plan)
    plan["cached"] = False
    return plan
