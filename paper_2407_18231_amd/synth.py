"""Seeded synthetic detector geometry and event generator.

This module only produces *inputs*: a module table describing an idealised
outer tracker made of double-sensor layers (each layer is two closely spaced
sensors, Sec. 1 of the paper), and events of helical tracks crossing it.
It holds none of the object-building arithmetic (no cuts, no windows, no
maps); the library and the oracle each derive those themselves from the
module table.

Geometry (all lengths in cm, field in T, momenta in GeV):

* barrel: six cylinders, mean radius R in (23, 36, 51, 68, 86, 110), sensors
  at R -/+ g/2 with g = 0.26 cm, split into phi sectors x z segments;
* endcap (PU200-like geometry only): five disks per side at |z| in
  (140, 165, 195, 230, 270), sensor planes at |z| -/+ g/2, r in [20, 110] in
  5 cm rings below r = 60 and 10 cm rings above, each ring split in phi.

Tracks are prompt helices in a uniform field along +z: vertex (0, 0, vz),
charge q = +/-1.  A positive charge turns clockwise (phi decreases along the
track).  Hits are the true crossings of each sensor on the outgoing branch
(turning angle below pi), smeared with a Gaussian truncated at 5 sigma.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

KAPPA_PER_T_GEV = 0.299792458e-2  # curvature [1/cm] = this * B[T] / pT[GeV]

BARREL_RADII = (23.0, 36.0, 51.0, 68.0, 86.0, 110.0)
SENSOR_GAP = 0.26
DISK_Z = (140.0, 165.0, 195.0, 230.0, 270.0)
DISK_RING_EDGES = (20.0, 25.0, 30.0, 35.0, 40.0, 45.0, 50.0, 55.0, 60.0,
                   70.0, 80.0, 90.0, 100.0, 110.0)

BARREL = 0
ENDCAP = 1


@dataclass
class Geometry:
    """Module table (one row per double-sensor module) plus lookup helpers.

    Row fields (numpy arrays of length n_mod):
      kind   : 0 barrel, 1 endcap
      layer  : barrel layer index 0..5, or disk index 0..4
      side   : 0 for barrel, +1 / -1 for the endcap at +z / -z
      s_lo, s_hi : lower / upper sensor position: radius (barrel) or signed
                   plane z (endcap); "lower" is the sensor nearer the
                   interaction point
      c_min, c_max : extent in the other coordinate: z (barrel), r (endcap)
      phi_min, phi_max : azimuth range [phi_min, phi_max) inside [0, 2 pi)
    """
    name: str
    kind: np.ndarray
    layer: np.ndarray
    side: np.ndarray
    s_lo: np.ndarray
    s_hi: np.ndarray
    c_min: np.ndarray
    c_max: np.ndarray
    phi_min: np.ndarray
    phi_max: np.ndarray
    # lookup: list of per-surface dicts used by the generator to find modules
    surfaces: list = field(default_factory=list)

    @property
    def n_mod(self) -> int:
        return int(self.kind.shape[0])

    def table(self) -> dict:
        return dict(kind=self.kind, layer=self.layer, side=self.side,
                    s_lo=self.s_lo, s_hi=self.s_hi, c_min=self.c_min,
                    c_max=self.c_max, phi_min=self.phi_min,
                    phi_max=self.phi_max)


def _build(name, barrel_specs, disk_specs):
    rows = {k: [] for k in ("kind", "layer", "side", "s_lo", "s_hi", "c_min",
                            "c_max", "phi_min", "phi_max")}
    surfaces = []
    base = 0
    for layer, (R, half, n_phi, n_z) in enumerate(barrel_specs):
        z_edges = np.linspace(-half, half, n_z + 1)
        surf = dict(kind=BARREL, layer=layer, side=0, base=base, n_phi=n_phi,
                    n_z=n_z, half=half, r_lo=R - SENSOR_GAP / 2,
                    r_hi=R + SENSOR_GAP / 2, z_edges=z_edges)
        for iz in range(n_z):
            for ip in range(n_phi):
                rows["kind"].append(BARREL)
                rows["layer"].append(layer)
                rows["side"].append(0)
                rows["s_lo"].append(R - SENSOR_GAP / 2)
                rows["s_hi"].append(R + SENSOR_GAP / 2)
                rows["c_min"].append(z_edges[iz])
                rows["c_max"].append(z_edges[iz + 1])
                rows["phi_min"].append(2 * math.pi * ip / n_phi)
                rows["phi_max"].append(2 * math.pi * (ip + 1) / n_phi)
        base += n_phi * n_z
        surfaces.append(surf)
    for side in (+1, -1):
        for disk, Z in enumerate(disk_specs["z"]):
            edges = np.asarray(disk_specs["rings"], dtype=np.float64)
            nphis = [int(math.ceil(2 * math.pi * 0.5 * (edges[i] + edges[i + 1]) / 10.0))
                     for i in range(len(edges) - 1)]
            ring_base = []
            b = base
            for n in nphis:
                ring_base.append(b)
                b += n
            surf = dict(kind=ENDCAP, layer=disk, side=side, base=base,
                        z_lo=side * (Z - SENSOR_GAP / 2),
                        z_hi=side * (Z + SENSOR_GAP / 2), ring_edges=edges,
                        ring_nphi=np.asarray(nphis), ring_base=np.asarray(ring_base))
            for ir, n in enumerate(nphis):
                for ip in range(n):
                    rows["kind"].append(ENDCAP)
                    rows["layer"].append(disk)
                    rows["side"].append(side)
                    rows["s_lo"].append(side * (Z - SENSOR_GAP / 2))
                    rows["s_hi"].append(side * (Z + SENSOR_GAP / 2))
                    rows["c_min"].append(edges[ir])
                    rows["c_max"].append(edges[ir + 1])
                    rows["phi_min"].append(2 * math.pi * ip / n)
                    rows["phi_max"].append(2 * math.pi * (ip + 1) / n)
            base = b
            surfaces.append(surf)
    g = Geometry(
        name=name,
        kind=np.asarray(rows["kind"], dtype=np.uint32),
        layer=np.asarray(rows["layer"], dtype=np.uint32),
        side=np.asarray(rows["side"], dtype=np.int32),
        s_lo=np.asarray(rows["s_lo"], dtype=np.float64),
        s_hi=np.asarray(rows["s_hi"], dtype=np.float64),
        c_min=np.asarray(rows["c_min"], dtype=np.float64),
        c_max=np.asarray(rows["c_max"], dtype=np.float64),
        phi_min=np.asarray(rows["phi_min"], dtype=np.float64),
        phi_max=np.asarray(rows["phi_max"], dtype=np.float64),
        surfaces=surfaces)
    return g


def make_geometry(name: str) -> Geometry:
    """'tiny': barrel only, 12 phi x 8 z modules per layer, half-length 170 cm
    (576 modules).  'pu200': barrel with ~10 cm phi modules, 5 cm (layers 1-3)
    or 10 cm (layers 4-6) z segments, half-length 130 cm, plus 2 x 5 disks
    (12 800 modules)."""
    if name == "tiny":
        specs = [(R, 170.0, 12, 8) for R in BARREL_RADII]
        return _build(name, specs, {"z": (), "rings": DISK_RING_EDGES})
    if name == "pu200":
        specs = []
        for i, R in enumerate(BARREL_RADII):
            n_phi = int(math.ceil(2 * math.pi * R / 10.0))
            n_z = 52 if i < 3 else 26
            specs.append((R, 130.0, n_phi, n_z))
        return _build(name, specs, {"z": DISK_Z, "rings": DISK_RING_EDGES})
    raise ValueError(f"unknown geometry {name!r}")


# --------------------------------------------------------------------------
# events
# --------------------------------------------------------------------------

@dataclass
class EventConfig:
    n_tracks: int = 50
    pt_mode: str = "uniform"        # "uniform" in [pt_lo, pt_hi], or "power": dN/dpT ~ pT^-3 above pt_lo
    pt_lo: float = 0.8
    pt_hi: float = 5.0
    eta_max: float = 1.0
    vz_sigma: float = 5.0
    B: float = 3.8
    sigma_rphi: float = 30e-4       # 30 um
    sigma_c: float = 0.1            # 1 mm (z in the barrel, r on the disks)
    smear: bool = True
    ineff: float = 0.0              # probability to drop a true hit
    noise_count: int = 0            # fixed number of noise hits ...
    noise_frac: float = 0.0         # ... or a fraction of the true-hit count
    n_pls: int = 0
    pls_fake_frac: float = 0.0
    pls_pt_min: float = 0.8
    pls_smear: bool = True
    # explicit track list (q, pt, eta, phi0, vz) overrides the random draw
    tracks: np.ndarray | None = None
    # displaced tracks added to the random draw: production radius uniform
    # in [0, rv_max] cm, pT uniform in [displaced_pt_lo, displaced_pt_hi],
    # |eta| < displaced_eta_max; no pixel seed is drawn from them
    n_displaced: int = 0
    rv_max: float = 35.0
    displaced_pt_lo: float = 1.0
    displaced_pt_hi: float = 10.0
    displaced_eta_max: float = 2.0


def config_tiny(**kw) -> EventConfig:
    """Tiny event: 50 tracks, pT U[0.8, 5], |eta| < 1, 200 noise hits."""
    c = EventConfig(n_tracks=50, pt_mode="uniform", pt_lo=0.8, pt_hi=5.0,
                    eta_max=1.0, noise_count=200)
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def config_pu(pu: float, noise_frac: float = 0.2, fake_frac: float = 0.02,
              **kw) -> EventConfig:
    """PU-like event: 20*PU tracks with dN/dpT ~ pT^-3 above 0.5 GeV,
    |eta| < 2.4, 10% hit inefficiency, noise_frac extra noise hits, 10*PU
    pixel seeds with fake_frac fakes."""
    c = EventConfig(n_tracks=int(round(20 * pu)), pt_mode="power", pt_lo=0.5,
                    eta_max=2.4, ineff=0.1, noise_frac=noise_frac,
                    n_pls=int(round(10 * pu)), pls_fake_frac=fake_frac)
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def _normal(rng, n, clip=5.0):
    return np.clip(rng.standard_normal(n), -clip, clip)


def draw_tracks(cfg: EventConfig, rng) -> np.ndarray:
    if cfg.tracks is not None:
        return np.asarray(cfg.tracks, dtype=np.float64).reshape(-1, 5)
    n = cfg.n_tracks
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    if cfg.pt_mode == "uniform":
        pt = rng.uniform(cfg.pt_lo, cfg.pt_hi, n)
    elif cfg.pt_mode == "power":
        u = rng.random(n)
        pt = cfg.pt_lo * (1.0 - u) ** -0.5
    else:
        raise ValueError(cfg.pt_mode)
    eta = rng.uniform(-cfg.eta_max, cfg.eta_max, n)
    phi0 = rng.uniform(0.0, 2 * math.pi, n)
    vz = rng.normal(0.0, cfg.vz_sigma, n)
    return np.stack([q, pt, eta, phi0, vz], axis=1)


def _module_of(geom: Geometry, surf: dict, phi, c):
    """Module id of points on a surface (phi in [0, 2pi), c = z or r); -1 if
    outside."""
    phi = np.mod(phi, 2 * math.pi)
    if surf["kind"] == BARREL:
        ze = surf["z_edges"]
        iz = np.searchsorted(ze, c, side="right") - 1
        ok = (iz >= 0) & (iz < surf["n_z"])
        ip = np.minimum((phi * surf["n_phi"] / (2 * math.pi)).astype(np.int64),
                        surf["n_phi"] - 1)
        mod = surf["base"] + iz * surf["n_phi"] + ip
    else:
        re = surf["ring_edges"]
        ir = np.searchsorted(re, c, side="right") - 1
        ok = (ir >= 0) & (ir < len(re) - 1)
        irc = np.clip(ir, 0, len(re) - 2)
        nph = surf["ring_nphi"][irc]
        ip = np.minimum((phi * nph / (2 * math.pi)).astype(np.int64), nph - 1)
        mod = surf["ring_base"][irc] + ip
    return np.where(ok, mod, -1)


def draw_displaced(cfg: EventConfig, rng):
    """Displaced tracks: (q, pT, eta, phi0, vz) as for prompt ones (phi0 the
    direction at the production point) and their production points: radius
    uniform in [0, rv_max], azimuth within 0.3 rad of the direction (the
    decay of a particle flying outward), z on the line from (0, 0, vz) along
    the track's polar direction."""
    n = cfg.n_displaced
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    pt = rng.uniform(cfg.displaced_pt_lo, cfg.displaced_pt_hi, n)
    eta = rng.uniform(-cfg.displaced_eta_max, cfg.displaced_eta_max, n)
    phi0 = rng.uniform(0.0, 2 * math.pi, n)
    vz = rng.normal(0.0, cfg.vz_sigma, n)
    rv = rng.uniform(0.0, cfg.rv_max, n)
    phv = phi0 + rng.uniform(-0.3, 0.3, n)
    vtx = np.stack([rv * np.cos(phv), rv * np.sin(phv), vz + rv * np.sinh(eta)], axis=1)
    return np.stack([q, pt, eta, phi0, vz], axis=1), vtx


def _crossings_displaced(surf: dict, sensor: int, q, pt, eta, phi0, vtx, B: float):
    """Sensor crossings of helices starting at vtx (x0, y0, z0) with
    direction phi0: the first crossing along the track of the barrel radius
    or disk plane, within half a turn."""
    kappa = KAPPA_PER_T_GEV * B / pt
    omega = -q * kappa
    cot = np.sinh(eta)
    x0, y0, z0 = vtx[:, 0], vtx[:, 1], vtx[:, 2]
    cx = x0 - np.sin(phi0) / omega           # centre of the transverse circle
    cy = y0 + np.cos(phi0) / omega
    half = math.pi / np.abs(omega)           # arc length of half a turn
    if surf["kind"] == BARREL:
        r = surf["r_lo"] if sensor == 0 else surf["r_hi"]
        # |P(s)|^2 = |C|^2 + R^2 + (2/omega)(cx sin u - cy cos u), u = phi0 + omega s
        c2 = cx * cx + cy * cy
        rad = 1.0 / (omega * omega)
        cn = np.sqrt(c2)
        with np.errstate(divide="ignore", invalid="ignore"):
            k = (r * r - c2 - rad) * omega / 2.0 / cn
        ok = np.abs(k) <= 1.0
        beta = np.arctan2(-cy, cx)             # cx sin u - cy cos u = cn sin(u + beta)
        a1 = np.arcsin(np.clip(k, -1.0, 1.0))
        s_best = np.full(q.shape, np.nan)
        for u in (a1 - beta, math.pi - a1 - beta):
            sv = np.mod((u - phi0) / omega, 2 * math.pi / np.abs(omega))
            sv = np.where(sv < 1e-9, np.nan, sv)
            s_best = np.fmin(s_best, sv)
        s = np.where(ok & (s_best <= half), s_best, np.nan)
        z = z0 + cot * s
        valid = np.isfinite(s) & (np.abs(z) <= surf["half"])
    else:
        zp = surf["z_lo"] if sensor == 0 else surf["z_hi"]
        with np.errstate(divide="ignore", invalid="ignore"):
            s = (zp - z0) / cot
        valid = (s > 0) & (s <= half)
        s = np.where(valid, s, np.nan)
        z = np.full_like(s, zp)
    u = phi0 + omega * s
    x = cx + np.sin(u) / omega
    y = cy - np.cos(u) / omega
    return valid, x, y, z, s


def propagate(geom: Geometry, trk: np.ndarray, B: float, vtx: np.ndarray | None = None):
    """True sensor crossings of helices: prompt ones (from (0, 0, vz)) and,
    for the tracks given production points vtx (rows of x0, y0, z0; NaN
    rows: prompt), displaced ones.

    Returns a list over (surface, sensor) of dicts with arrays over tracks:
    valid mask, x, y, z, phi, r, s (transverse arc length), module id."""
    q, pt, eta, phi0, vz = (trk[:, i] for i in range(5))
    kappa = KAPPA_PER_T_GEV * B / pt
    omega = -q * kappa                      # dphi/ds
    cot = np.sinh(eta)
    disp = np.zeros(q.shape, bool) if vtx is None else np.isfinite(vtx[:, 0])
    out = []
    for surf in geom.surfaces:
        for sensor in (0, 1):
            if surf["kind"] == BARREL:
                r = surf["r_lo"] if sensor == 0 else surf["r_hi"]
                arg = r * kappa / 2.0
                reach = arg <= 1.0
                s = np.where(reach, 2.0 / kappa * np.arcsin(np.minimum(arg, 1.0)), np.nan)
                z = vz + cot * s
                valid = reach & (np.abs(z) <= surf["half"])
                rr = np.full_like(s, r)
                c = z
            else:
                zp = surf["z_lo"] if sensor == 0 else surf["z_hi"]
                with np.errstate(divide="ignore", invalid="ignore"):
                    s = (zp - vz) / cot
                valid = (s > 0) & (kappa * s < math.pi)
                s = np.where(valid, s, np.nan)
                rr = 2.0 / kappa * np.sin(kappa * s / 2.0)
                z = np.full_like(s, zp)
                c = rr
            phi = phi0 + omega * s / 2.0
            x = rr * np.cos(phi)
            y = rr * np.sin(phi)
            if disp.any():
                dv, dx, dy, dz, ds = _crossings_displaced(surf, sensor, q[disp], pt[disp], eta[disp],
                                                         phi0[disp], vtx[disp], B)
                valid = valid.copy()
                valid[disp] = dv
                x = x.copy(); y = y.copy(); z = z.copy(); s = s.copy()
                x[disp], y[disp], z[disp], s[disp] = dx, dy, dz, ds
                rr = np.hypot(x, y)
                phi = np.arctan2(y, x)
                c = z if surf["kind"] == BARREL else rr
            mod = np.full(s.shape, -1, dtype=np.int64)
            if valid.any():
                mod[valid] = _module_of(geom, surf, phi[valid], c[valid])
            valid = valid & (mod >= 0)
            out.append(dict(surf=surf, sensor=sensor, valid=valid, x=x, y=y,
                            z=z, r=rr, phi=phi, s=s, module=mod))
    return out


def _module_areas(geom: Geometry):
    dphi = geom.phi_max - geom.phi_min
    barrel = geom.kind == BARREL
    area = np.where(barrel,
                    0.5 * (geom.s_lo + geom.s_hi) * dphi * (geom.c_max - geom.c_min),
                    0.5 * (geom.c_max ** 2 - geom.c_min ** 2) * dphi)
    return area


def gen_event(geom: Geometry, cfg: EventConfig, seed: int) -> dict:
    """One synthetic event.

    Returns dict with
      x, y, z (float32), module (uint32), sensor (uint8): hits in a random
        order (the caller-visible input order);
      hit_track (int32): generating track of each hit, -1 for noise;
      pls_par (float32 [n,5]: q/pT, phi0, cot(theta), d0, z0),
      pls_cov (float32 [n,15]: upper triangle of the 5x5 covariance, row
        major), pls_track (int32, -1 for fakes), pls_nhits (uint8: pixel
        hits of each seed, 3 or 4);
      tracks (float64 [n,5]: q, pT, eta, phi0, vz), track_rv (float64 [n]:
        production radius, 0 for prompt tracks).
    """
    rng = np.random.default_rng(seed)
    trk = draw_tracks(cfg, rng)
    vtx = None
    if cfg.n_displaced:
        dtrk, dvtx = draw_displaced(cfg, rng)
        vtx = np.concatenate([np.full((trk.shape[0], 3), np.nan), dvtx])
        trk = np.concatenate([trk, dtrk])
    n_trk = trk.shape[0]
    cr = propagate(geom, trk, cfg.B, vtx)
    xs, ys, zs, mods, sens, tids = [], [], [], [], [], []
    for c in cr:
        v = c["valid"].copy()
        if cfg.ineff > 0:
            v &= rng.random(n_trk) >= cfg.ineff
        idx = np.nonzero(v)[0]
        if idx.size == 0:
            continue
        x = c["x"][idx].copy()
        y = c["y"][idx].copy()
        z = c["z"][idx].copy()
        phi = c["phi"][idx]
        if cfg.smear:
            d_t = cfg.sigma_rphi * _normal(rng, idx.size)
            x += -np.sin(phi) * d_t
            y += np.cos(phi) * d_t
            if c["surf"]["kind"] == BARREL:
                z += cfg.sigma_c * _normal(rng, idx.size)
            else:
                d_r = cfg.sigma_c * _normal(rng, idx.size)
                x += np.cos(phi) * d_r
                y += np.sin(phi) * d_r
        xs.append(x); ys.append(y); zs.append(z)
        mods.append(c["module"][idx]); sens.append(np.full(idx.size, c["sensor"]))
        tids.append(idx)
    n_true = int(sum(a.size for a in xs))
    n_noise = cfg.noise_count if cfg.noise_count else int(round(cfg.noise_frac * n_true))
    if n_noise > 0:
        area = _module_areas(geom)
        p = area / area.sum()
        m = rng.choice(geom.n_mod, size=n_noise, p=p)
        sensor = (rng.random(n_noise) < 0.5).astype(np.int64)
        phi = rng.uniform(geom.phi_min[m], geom.phi_max[m])
        barrel = geom.kind[m] == BARREL
        pos = np.where(sensor == 0, geom.s_lo[m], geom.s_hi[m])
        zc = rng.uniform(geom.c_min[m], geom.c_max[m])
        u = rng.random(n_noise)
        rc = np.sqrt(np.abs(geom.c_min[m] ** 2 + u * (geom.c_max[m] ** 2 - geom.c_min[m] ** 2)))
        r = np.where(barrel, pos, rc)
        z = np.where(barrel, zc, pos)
        xs.append(r * np.cos(phi)); ys.append(r * np.sin(phi)); zs.append(z)
        mods.append(m); sens.append(sensor); tids.append(np.full(n_noise, -1))
    if xs:
        x = np.concatenate(xs); y = np.concatenate(ys); z = np.concatenate(zs)
        mod = np.concatenate(mods); sen = np.concatenate(sens)
        tid = np.concatenate(tids)
    else:
        x = y = z = np.zeros(0); mod = sen = tid = np.zeros(0, dtype=np.int64)
    perm = rng.permutation(x.size)
    ev = dict(x=x[perm].astype(np.float32), y=y[perm].astype(np.float32),
              z=z[perm].astype(np.float32), module=mod[perm].astype(np.uint32),
              sensor=sen[perm].astype(np.uint8), hit_track=tid[perm].astype(np.int32),
              tracks=trk)
    rv = np.zeros(n_trk) if vtx is None else np.where(np.isfinite(vtx[:, 0]), np.hypot(vtx[:, 0], vtx[:, 1]), 0.0)
    ev["track_rv"] = rv
    par, cov, ptid = gen_pls(trk, cfg, rng, prompt=rv == 0.0)
    ev.update(pls_par=par, pls_cov=cov, pls_track=ptid, pls_nhits=seed_pixel_hits(ptid, seed))
    return ev


def seed_pixel_hits(pls_track: np.ndarray, seed: int) -> np.ndarray:
    """Pixel hits of each seed: 4 (a quad) with probability 0.7 for a seed
    from a track and 0.4 for a fake, else 3 (a triplet); drawn from a
    generator of its own, so the rest of the event does not depend on it."""
    rng = np.random.default_rng([seed, 0x5EED])
    p_quad = np.where(pls_track >= 0, 0.7, 0.4)
    return np.where(rng.random(pls_track.size) < p_quad, 4, 3).astype(np.uint8)


def gen_pls(trk: np.ndarray, cfg: EventConfig, rng, prompt: np.ndarray | None = None):
    """Pixel seeds: helix parameters plus covariance.  True seeds are drawn
    with replacement from tracks above pls_pt_min; fakes combine values drawn
    independently from the true seeds' marginals."""
    n = cfg.n_pls
    par = np.zeros((n, 5), dtype=np.float64)
    tid = np.full(n, -1, dtype=np.int32)
    if n == 0:
        return par.astype(np.float32), np.zeros((0, 15), np.float32), tid
    ok = trk[:, 1] > cfg.pls_pt_min
    cand = np.nonzero(ok if prompt is None else ok & prompt)[0]
    n_fake = int(round(cfg.pls_fake_frac * n)) if cand.size else n
    n_true = n - n_fake
    sel = rng.choice(cand, size=n_true, replace=True) if n_true else np.zeros(0, np.int64)
    q, pt, eta, phi0, vz = (trk[sel, i] for i in range(5))
    qpt = q / pt
    cot = np.sinh(eta)
    s = lambda m: (_normal(rng, m) if cfg.pls_smear else np.zeros(m))
    t = np.empty((n_true, 5))
    t[:, 0] = qpt * (1.0 + 0.015 * s(n_true))
    t[:, 1] = phi0 + 1e-3 * s(n_true)
    t[:, 2] = cot + 2e-3 * s(n_true)
    t[:, 3] = 0.005 * s(n_true)
    t[:, 4] = vz + 0.01 * s(n_true)
    par[:n_true] = t
    tid[:n_true] = sel
    if n_fake:
        src = t if n_true else np.column_stack([
            trk[:, 0] / trk[:, 1], trk[:, 3], np.sinh(trk[:, 2]),
            np.zeros(trk.shape[0]), trk[:, 4]])
        for k in range(5):
            par[n_true:, k] = src[rng.integers(0, src.shape[0], n_fake), k]
        par[n_true:, 1] = rng.uniform(0.0, 2 * math.pi, n_fake)
    par[:, 1] = np.mod(par[:, 1], 2 * math.pi)
    cov = np.zeros((n, 15), dtype=np.float64)
    cov[:, 0] = (0.015 * par[:, 0]) ** 2
    cov[:, 5] = 1e-3 ** 2
    cov[:, 9] = 2e-3 ** 2
    cov[:, 12] = 0.005 ** 2
    cov[:, 14] = 0.01 ** 2
    order = rng.permutation(n)
    return (par[order].astype(np.float32), cov[order].astype(np.float32),
            tid[order])


# Event i of configuration c uses seed 1000*c + i.
def event_seed(config_index: int, i: int) -> int:
    return 1000 * config_index + i


def standard_event(kind: str, i: int = 0, geom: Geometry | None = None):
    """Workloads used by tests and the benchmark.

    'tiny'   : tiny barrel event (config index 1)
    'pu200'  : single PU200-like event (config index 2)
    'pu300'  : stress PU300-like event, 40% noise, 5% fake seeds (index 5)
    """
    if kind == "tiny":
        g = geom or make_geometry("tiny")
        return g, gen_event(g, config_tiny(), event_seed(1, i))
    if kind == "pu200":
        g = geom or make_geometry("pu200")
        return g, gen_event(g, config_pu(200), event_seed(2, i))
    if kind == "pu300":
        g = geom or make_geometry("pu200")
        return g, gen_event(g, config_pu(300, noise_frac=0.4, fake_frac=0.05),
                            event_seed(5, i))
    raise ValueError(kind)


def batch_events(n: int, geom: Geometry, pu_lo=50.0, pu_hi=250.0, seed_base=3):
    """Mixed-pileup batch: PU ~ U[pu_lo, pu_hi] per event (config index 3)."""
    evs = []
    for i in range(n):
        rng = np.random.default_rng(event_seed(seed_base, i) + 500_000)
        pu = float(rng.uniform(pu_lo, pu_hi))
        evs.append(gen_event(geom, config_pu(pu), event_seed(seed_base, i)))
    return evs
