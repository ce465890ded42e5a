"""Pins of the synthetic input generator (helix geometry, determinism,
spectra).  The generator is the source of truth for the oracle pins, so it is
itself checked against closed forms here."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2407_18231_amd import synth as s


def test_geometry_module_counts():
    assert s.make_geometry("tiny").n_mod == 576
    g = s.make_geometry("pu200")
    assert g.n_mod == 12800
    assert int((g.kind == s.BARREL).sum()) == 8060
    # every module's extents are ordered and inside [0, 2 pi)
    assert np.all(g.c_max > g.c_min) and np.all(g.phi_max > g.phi_min)
    assert g.phi_min.min() >= 0 and g.phi_max.max() <= 2 * math.pi + 1e-12
    # lower sensor nearer the interaction point
    assert np.all(np.abs(g.s_lo) < np.abs(g.s_hi))


def test_hits_lie_on_helix_circle():
    """Noiseless hits of a track lie on the circle of radius pT/(0.3 B)
    through the origin whose centre is (-sin phi0, cos phi0)/omega with
    omega = -q kappa (a positive charge turns clockwise)."""
    g = s.make_geometry("pu200")
    cfg = s.config_pu(50, noise_frac=0.0, fake_frac=0.0, smear=False, ineff=0.0)
    ev = s.gen_event(g, cfg, 11)
    trk = ev["tracks"]
    t = ev["hit_track"]
    ok = t >= 0
    q, pt, eta, phi0, vz = (trk[t[ok], i] for i in range(5))
    kappa = s.KAPPA_PER_T_GEV * 3.8 / pt
    omega = -q * kappa
    cx, cy = -np.sin(phi0) / omega, np.cos(phi0) / omega
    x = ev["x"][ok].astype(np.float64); y = ev["y"][ok].astype(np.float64)
    R = np.hypot(x - cx, y - cy)
    assert np.max(np.abs(R * kappa - 1.0)) < 2e-5
    # z = vz + cot(theta) * s with s the transverse arc from the origin
    r = np.hypot(x, y)
    arc = 2.0 / kappa * np.arcsin(np.minimum(r * kappa / 2, 1.0))
    zp = vz + np.sinh(eta) * arc
    well = r * kappa / 2 < 0.9      # away from the turning point, where asin is ill-conditioned
    assert np.max(np.abs(zp - ev["z"][ok])[well]) < 5e-4
    # positive charges turn clockwise: phi of the hit lags phi0
    dphi = np.angle(np.exp(1j * (np.arctan2(y, x) - phi0)))
    assert np.all(np.sign(dphi[q > 0]) < 0) and np.all(np.sign(dphi[q < 0]) > 0)


def test_deterministic_per_seed():
    g = s.make_geometry("pu200")
    a = s.gen_event(g, s.config_pu(20), 5)
    b = s.gen_event(g, s.config_pu(20), 5)
    c = s.gen_event(g, s.config_pu(20), 6)
    for k in ("x", "y", "z", "module", "sensor", "pls_par", "pls_cov"):
        assert np.array_equal(a[k], b[k])
    assert not np.array_equal(a["x"][:10], c["x"][:10])


def test_pt_spectrum_power_law():
    rng = np.random.default_rng(3)
    cfg = s.config_pu(100)
    trk = s.draw_tracks(cfg, rng)
    pt = trk[:, 1]
    # P(pT < x) = 1 - (0.5/x)^2 for dN/dpT ~ pT^-3 above 0.5 GeV
    res = stats.kstest(pt, lambda x: 1.0 - (0.5 / np.maximum(x, 0.5)) ** 2)
    assert res.pvalue > 1e-3
    assert np.all(np.abs(trk[:, 2]) <= 2.4)


def test_pu200_sizes():
    g, ev = s.standard_event("pu200")
    n = ev["x"].size
    assert 45_000 < n < 65_000
    assert ev["pls_par"].shape == (2000, 5) and ev["pls_cov"].shape == (2000, 15)
    assert int((ev["pls_track"] < 0).sum()) == 40
    assert ev["module"].max() < g.n_mod and set(np.unique(ev["sensor"])) <= {0, 1}
