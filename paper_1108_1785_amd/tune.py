"""Autotuning cache for the batched form.

gnm_autotune (C ABI) times launch shapes on the caller's own records; this
module remembers the winner in a JSON file keyed by device, library version,
registry shape and workload size, so later runs of the same workload skip the
search.  The cache holds launch parameters only, never results.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Optional

from . import Registry, autotune, lib, version

DEFAULT_CACHE = os.path.join(os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")), "gnm", "tune.json")


def _cache_path() -> str:
    return os.environ.get("GNM_TUNE_CACHE", DEFAULT_CACHE)


def _device_name() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return "%s/%s/%d" % (p.name, getattr(p, "gcnArchName", ""), p.multi_processor_count)


def workload_key(reg: Registry, n_records: int, n_windows: int, workspace_bytes: int = 0) -> str:
    i = reg.info()
    shape = "p%d-s%d-r%d-l%d-li%d-ai%d" % (i["n_prefixes"], i["n_sites"], i["root_bits"], i["list_max"],
                                          i["lines_in_lds"], i["acc_in_lds"])
    # sizes bucketed by powers of two: the best shape changes slowly with size
    nb = int(math.log2(max(n_records, 1)))
    wb = int(math.log2(max(n_windows, 1)))
    # the merge path: atomics, or the workspace (partial tables, or the
    # spilled rows of a table beyond LDS) for shapes up to the workgroup count
    # the workspace holds (candidates beyond it are not timed)
    g = max_grid_for(reg, workspace_bytes, n_records, n_windows) if workspace_bytes else 0
    merge = "atomic" if not g else ("ws%d" if i["acc_in_lds"] else "spill%d") % g
    return "%s|%s|%s|n2^%d|w2^%d|%s" % (_device_name(), version(), shape, nb, wb, merge)


def max_grid_for(reg: Registry, workspace_bytes: int, n_records: int = 0, n_windows: int = 1) -> int:
    """Largest tuning candidate workgroup count whose workspace fits workspace_bytes (0: none)."""
    best = 0
    for g in candidate_grids(reg):
        need = workspace_bytes_for(reg, g, n_records, n_windows)
        if need and need <= workspace_bytes:
            best = max(best, g)
    return best


def _resident(reg: Registry) -> int:
    import torch
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    return cus * (2 if reg.info()["lds_bytes"] <= 80 * 1024 else 1)


def candidate_grids(reg: Registry):
    """Workgroup counts gnm_autotune tries (the automatic count is the resident one)."""
    r = _resident(reg)
    return [r, r // 2, 2 * r, 4 * r]


def workspace_bytes_for(reg: Registry, grid: int, n_records: int = 0, n_windows: int = 1) -> int:
    from . import workspace_bytes_n
    return workspace_bytes_n(reg, n_records, n_windows, grid)


def tuning_workspace(reg: Registry, device=None, n_records: int = 0, n_windows: int = 1):
    """A workspace large enough for every tuning candidate, so all of them
    are timed on the merge that the tuned launch uses (the partial tables, or,
    for a table beyond LDS, the spilled rows of n_records records)."""
    from . import make_workspace
    return make_workspace(reg, max(candidate_grids(reg)), device=device, n_records=n_records, n_windows=n_windows)


def _load(path: str) -> Dict[str, dict]:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, data: Dict[str, dict]) -> None:
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only cache only costs a re-tune


def tuned_params(reg: Registry, rec, acc, window_offsets=None, n_windows: int = 1, n: Optional[int] = None,
                 workspace=None, reps: int = 3, refresh: bool = False,
                 cache_path: Optional[str] = None) -> Dict[str, object]:
    """{"records_per_thread", "grid_blocks", ...} for this workload, tuned once and cached."""
    lib()
    path = cache_path or _cache_path()
    n_rec = int(n if n is not None else rec["src_ip"].numel())
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    key = workload_key(reg, n_rec, n_windows, ws_bytes)
    data = _load(path)
    if not refresh and key in data:
        hit = dict(data[key])
        hit["cached"] = True
        return hit
    res = autotune(reg, rec, acc, window_offsets=window_offsets, n_windows=n_windows, reps=reps, n=n_rec,
                   workspace=workspace)
    entry = {"records_per_thread": res["records_per_thread"], "grid_blocks": res["grid_blocks"],
             "best_ms": res["best_ms"], "tried": res["tried"]}
    data[key] = entry
    _store(path, data)
    out = dict(entry)
    out["cached"] = False
    return out
