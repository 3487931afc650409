"""The named workloads (patterns with their sizes), built deterministically.

* ``band200``     band pattern, n = 200, half-bandwidth 5.
* ``grid2d_128``  filled 2D 5-point grid 128 x 128 under geometric ND (n = 16384).
* ``arrow64``     block-arrow: 64 dense diagonal blocks of size uniform in
                  [32, 256] (``default_rng(0).integers(32, 257, 64)``) plus a
                  dense arrow of 128 rows (n = 9486).
* ``grid3d_40``   filled 3D 7-point grid 40^3 under geometric ND (n = 64000).
* ``er<n>_<seed>`` filled Erdos-Renyi graph, average degree 6, minimum degree.

Small variants (``grid2d_<s>``, ``grid3d_<s>``, ``band<n>``) serve tests.
"""
from __future__ import annotations

import functools
import re

from . import patterns

CONFIG_NAMES = ("band200", "grid2d_128", "arrow64", "grid3d_40")


@functools.lru_cache(maxsize=16)
def get_config(name: str):
    m = re.fullmatch(r"band(\d+)(?:_w(\d+))?", name)
    if m:
        return patterns.band(int(m.group(1)), int(m.group(2) or 5))
    m = re.fullmatch(r"grid2d_(\d+)", name)
    if m:
        s = int(m.group(1))
        return patterns.grid_nd((s, s))
    m = re.fullmatch(r"grid3d_(\d+)", name)
    if m:
        s = int(m.group(1))
        return patterns.grid_nd((s, s, s))
    if name == "arrow64":
        return patterns.block_arrow_config(0)
    m = re.fullmatch(r"arrow(\d+)_(\d+)_(\d+)_(\d+)", name)
    if m:
        nb, lo, hi, ar = (int(g) for g in m.groups())
        return patterns.block_arrow_config(0, nb, lo, hi, ar)
    m = re.fullmatch(r"er(\d+)_(\d+)", name)
    if m:
        return patterns.er_min_degree(int(m.group(1)), int(m.group(2)))
    raise KeyError(name)
