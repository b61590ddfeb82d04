"""Autotuner front end: picks the execution strategy (unfused, LDS tile
runs and their tile size, fused k = 2..5), the matrix-core kernel's tile
shape and its workgroups per CU for a circuit family by timing them with qc_autotune, and
caches the choice in a JSON file keyed by device, qubit count, element type
and circuit signature.

The cache path is $QC_TUNE_CACHE, else ~/.cache/qc_tune.json.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Optional

import torch

from . import qc

MODE_NAMES = {qc.QC_EXEC_UNFUSED: "unfused", qc.QC_EXEC_FUSED: "fused", qc.QC_EXEC_TILED: "tiled"}


def cache_path() -> str:
    return os.environ.get("QC_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "qc_tune.json"))


def circuit_key(n: int, dtype: torch.dtype, gate_tuples, family: Optional[str] = None) -> str:
    """Device + size + type + structure (targets and controls, not values)."""
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    if family is None:
        h = hashlib.sha1()
        for t, c, cv, _ in gate_tuples:
            h.update(repr((tuple(t), tuple(c), tuple(cv))).encode())
        family = h.hexdigest()[:16]
    return "%s|n=%d|%s|%s" % (dev, n, str(dtype).replace("torch.", ""), family)


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: dict) -> None:
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def tune(n: int, dtype: torch.dtype, gate_tuples, family: Optional[str] = None,
         reps: int = 3, force: bool = False) -> dict:
    """Best configuration for this circuit family (from the cache when
    present).  Tuning runs on a scratch state of the same size."""
    key = circuit_key(n, dtype, gate_tuples, family)
    cache = _load()
    if key in cache and not force:
        return cache[key]
    scratch = qc.new_state(n, dtype)
    saved = {k: qc.get_knob(k) for k in _KNOBS}
    try:
        table = qc.autotune(scratch, qc.GateList(gate_tuples), reps=reps)
    finally:
        # qc_autotune leaves the knobs at the winner's values; apply_tuned
        # sets them per call instead
        for k, v in saved.items():
            qc.set_knob(k, v)
    del scratch
    best = dict(table[0])
    best["mode_name"] = MODE_NAMES.get(best["mode"], str(best["mode"]))
    best["table"] = table
    cache[key] = best
    _store(cache)
    return best


_KNOBS = (qc.QC_KNOB_MFMA_WG_PER_CU, qc.QC_KNOB_MFMA_TILE_BITS, qc.QC_KNOB_TILE_BITS)


def apply_tuned(psi: torch.Tensor, gate_tuples, family: Optional[str] = None) -> dict:
    """Apply a circuit with its tuned configuration.  The launch-shape knobs
    are process-wide: they are set for this call only and restored after
    it, so later calls on other circuit families keep their own shapes."""
    n = qc.state_view(psi).n
    cfg = tune(n, psi.dtype, gate_tuples, family)
    saved = {k: qc.get_knob(k) for k in _KNOBS}
    try:
        if cfg["mode"] == qc.QC_EXEC_FUSED and cfg.get("mfma_wg_per_cu"):
            qc.set_knob(qc.QC_KNOB_MFMA_WG_PER_CU, cfg["mfma_wg_per_cu"])
        if cfg["mode"] == qc.QC_EXEC_FUSED and cfg.get("mfma_tile_bits") in (12, 13):
            qc.set_knob(qc.QC_KNOB_MFMA_TILE_BITS, cfg["mfma_tile_bits"])
        if cfg["mode"] == qc.QC_EXEC_TILED and cfg.get("tile_bits"):
            qc.set_knob(qc.QC_KNOB_TILE_BITS, cfg["tile_bits"])
        return qc.apply_circuit(psi, qc.GateList(gate_tuples), mode=cfg["mode"],
                                fuse_k=cfg["fuse_k"] or 5)
    finally:
        for k, v in saved.items():
            qc.set_knob(k, v)
