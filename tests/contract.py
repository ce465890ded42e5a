"""Module tables with shrunk extents (test helper for the input contract).

A hit that lies inside its module on geometry g lies, on ``shrunk(g, k)``,
at most k resolutions outside its module's extent: the azimuth range loses
k sig_rphi over the module's inner radius at each end, the z (barrel) or r
(endcap) range k sig_c at each end; sensor positions are unchanged.  Events
generated without smearing on g therefore probe the edge of the contract on
the shrunk table (k just below the accepted 5.5 resolutions) or break it
(k well above).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from paper_2407_18231_amd.synth import BARREL


def shrunk(geom, k: float, sig_rphi: float = 30e-4, sig_c: float = 0.1):
    barrel = geom.kind == BARREL
    c_min = geom.c_min + k * sig_c
    c_max = geom.c_max - k * sig_c
    r_min = np.where(barrel, geom.s_lo, c_min)
    dphi = k * sig_rphi / r_min
    return dataclasses.replace(geom, name=f"{geom.name}-shrunk{k}", c_min=c_min, c_max=c_max,
                               phi_min=geom.phi_min + dphi, phi_max=geom.phi_max - dphi)


def outside_extent(geom, ev, sig_rphi: float = 30e-4, sig_c: float = 0.1) -> np.ndarray:
    """How far (in resolutions) each hit lies outside its module's extent
    (0 inside), in binary64, for the coarse coordinate and the azimuth."""
    m = ev["module"].astype(np.int64)
    x, y, z = (ev[k].astype(np.float64) for k in ("x", "y", "z"))
    r = np.hypot(x, y)
    barrel = geom.kind[m] == BARREL
    c = np.where(barrel, z, r)
    dc = np.maximum(geom.c_min[m] - c, c - geom.c_max[m]).clip(min=0) / sig_c
    phi = np.mod(np.arctan2(y, x), 2 * np.pi)
    lo, hi = geom.phi_min[m], geom.phi_max[m]
    cen = 0.5 * (lo + hi)
    d = np.abs(np.mod(phi - cen + np.pi, 2 * np.pi) - np.pi)
    r_min = np.where(barrel, geom.s_lo[m], geom.c_min[m])
    dp = (d - 0.5 * (hi - lo)).clip(min=0) * r_min / sig_rphi
    return np.maximum(dc, dp)
