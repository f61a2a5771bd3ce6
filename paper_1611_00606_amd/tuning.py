"""Tile-shape tuning of the batched per-atom stage.

`autotune` measures every batched tile shape per N_L on the current device
(hs_autotune_atoms in the library does the timing) and returns the hs_tuning
table to pass as `tuning=` to hs_build_ex / DeviceBuild / Context.build. A
JSON cache file keyed by device architecture, N_G and N_L keeps the chosen
shape (as "BMxBN") across processes, so the measurement runs once per N_L.
"""

from __future__ import annotations

import json
import os
from typing import Dict, Iterable, Optional, Tuple

from . import _binding as B


def _arch() -> str:
    import torch
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def tuning_from_table(table: Dict[int, int]) -> B.hs_tuning:
    """hs_tuning from {N_L: shape id}; other N_L keep the built-in choice."""
    t = B.hs_tuning()
    for v in range(B.HS_MAX_NL + 1):
        t.cfg[v] = default_shape(v)
    for v, c in table.items():
        if not 1 <= int(v) <= B.HS_MAX_NL or B.hs_tile_config(int(c)) is None:
            raise ValueError(f"bad tuning entry {v}: {c}")
        t.cfg[int(v)] = int(c)
    return t


def default_shape(nl: int) -> int:
    """The library's built-in shape id for N_L (used when no table is given):
    the tile with the fewest rows (32, 64, 96, 128) covering N_L, 128 columns
    wide except for 96 rows (192 columns)."""
    return 0 if nl <= 32 else 1 if nl <= 64 else 6 if nl <= 96 else 3


def _shape_id(bm_bn: str) -> Optional[int]:
    """Shape id of a cached "BMxBN" entry, or None when the library has no
    such shape (a cache written for another shape set is measured again)."""
    for c, s in shapes().items():
        if isinstance(bm_bn, str) and bm_bn == f"{s[0]}x{s[1]}":
            return c
    return None


def autotune(nl_values: Iterable[int], n_g: int, reps: int = 3,
             cache: Optional[str] = None) -> Tuple[B.hs_tuning, Dict[int, Dict]]:
    """Fastest shape per N_L at n_g columns.

    Returns (tuning, report) where report[N_L] = {"shape": id, "bm_bn": (BM, BN),
    "ms": [time per shape] or None when the entry came from the cache}."""
    vals = sorted({int(v) for v in nl_values})
    key_base = f"{_arch()}/N_G={int(n_g)}"
    stored = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            stored = json.load(f)
    table, report, todo = {}, {}, []
    for v in vals:
        k = f"{key_base}/N_L={v}"
        c = _shape_id(stored.get(k))
        if c is not None:
            table[v] = c
            report[v] = {"shape": c, "bm_bn": B.hs_tile_config(c), "ms": None}
        else:
            todo.append(v)
    if todo:
        t, ms = B.hs_autotune_atoms(todo, n_g, reps)
        for i, v in enumerate(todo):
            table[v] = int(t.cfg[v])
            report[v] = {"shape": table[v], "bm_bn": B.hs_tile_config(table[v]),
                         "ms": [round(float(x), 4) for x in ms[i]]}
            bm, bn = B.hs_tile_config(table[v])
            stored[f"{key_base}/N_L={v}"] = f"{bm}x{bn}"
        if cache:
            d = os.path.dirname(os.path.abspath(cache))
            os.makedirs(d, exist_ok=True)
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(stored, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
    return tuning_from_table(table), report


def shapes() -> Dict[int, Tuple[int, int]]:
    """All batched tile shapes: id -> (BM, BN)."""
    return {c: B.hs_tile_config(c) for c in range(B.HS_NUM_TILE_CONFIGS)}


__all__ = ["autotune", "tuning_from_table", "default_shape", "shapes"]
