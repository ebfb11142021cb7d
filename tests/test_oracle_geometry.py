"""Pins of the oracle's geometry generality (the layer description of
Section 2.1): stereo layers, whose hits measure in a turned strip frame, and
layers with a hole without sensors.  Against the strip-frame chi2 and Kalman
update written with the rotation on the other side, the hole's edges, and a
find on the CMS-like geometry.  CPU only."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import BARREL, DISK, FindConfig, Layer, cms_like, generate_event

BZ = 3.8


def random_psd(rng, scale):
    A = rng.normal(size=(6, 6)) * scale
    return A @ A.T


def state_on(kind, rng):
    if kind == BARREL:
        a = rng.uniform(-np.pi, np.pi)
        return np.array([25 * np.cos(a), 25 * np.sin(a), rng.uniform(-50, 50), 0.5, a + 0.1, 1.2])
    a = rng.uniform(-np.pi, np.pi)
    r = rng.uniform(30, 90)
    return np.array([r * np.cos(a), r * np.sin(a), 150.0, 0.5, a + 0.1, 0.4])


def hit_near(p, kind, rng):
    h = p[:3].copy()
    if kind == BARREL:
        a = np.arctan2(p[1], p[0]) + rng.normal(0, 1e-3)
        r = np.hypot(p[0], p[1])
        h[0], h[1] = r * np.cos(a), r * np.sin(a)
        h[2] += rng.normal(0, 0.3)
    else:
        h[0] += rng.normal(0, 0.05)
        h[1] += rng.normal(0, 0.05)
    return h


@pytest.mark.parametrize("kind", [BARREL, DISK])
def test_stereo_chi2_equals_the_strip_frame_chi2(kind):
    """chi2 with the covariance turned into (u, v) equals the chi2 of the
    residual and the prediction turned into the strip frame, where the hit
    covariance is diagonal."""
    rng = np.random.default_rng(71)
    for _ in range(20):
        p = state_on(kind, rng)
        Cm = random_psd(rng, 0.02)
        h = hit_near(p, kind, rng)
        a, vw, vp = rng.uniform(-0.5, 0.5), 1e-5, rng.uniform(0.01, 1.0)
        got = O.chi2(p, Cm, kind, h, vw, vp, a)
        ok, r, H = O.measure(p, kind, h)
        R = np.array([[np.cos(a), np.sin(a)], [-np.sin(a), np.cos(a)]])
        rs, Hs = R @ r, R @ H
        S = Hs @ Cm @ Hs.T + np.diag([vw, vp])
        want = rs @ np.linalg.solve(S, rs)
        assert got == pytest.approx(want, rel=1e-9)


@pytest.mark.parametrize("kind", [BARREL, DISK])
def test_stereo_update_equals_the_strip_frame_update(kind):
    """The Kalman update with the turned hit covariance equals the update
    with the measurement turned into the strip frame (general update,
    rotated H and r, diagonal V)."""
    rng = np.random.default_rng(72)
    for _ in range(20):
        p = state_on(kind, rng)
        Cm = random_psd(rng, 0.02)
        h = hit_near(p, kind, rng)
        a, vw, vp = rng.uniform(-0.5, 0.5), 1e-5, rng.uniform(0.01, 1.0)
        ok, p1, C1, c2 = O.update_hit(p, Cm, kind, h, vw, vp, a)
        assert ok
        _, r, H = O.measure(p, kind, h)
        R = np.array([[np.cos(a), np.sin(a)], [-np.sin(a), np.cos(a)]])
        p2, C2, c22 = O.kf_update(p, Cm, R @ H, R @ r, np.diag([vw, vp]).ravel())
        d = p1 - p2
        d[4] = np.arctan2(np.sin(d[4]), np.cos(d[4]))
        assert np.allclose(d, 0, atol=1e-10 * (1 + np.abs(p2).max()))
        assert np.allclose(C1, C2, rtol=1e-7, atol=1e-12)
        assert c2 == pytest.approx(c22, rel=1e-9)


@pytest.mark.parametrize("kind", [BARREL, DISK])
def test_hole_edges(kind):
    """A crossing inside a layer's hole (shrunk by the edge margin) is
    outside the layer; one outside the hole is on it."""
    fc = FindConfig()
    if kind == BARREL:
        lay = Layer(BARREL, 25.0, -100, 100, 1e-5, 1e-4, hole_lo=-2.0, hole_hi=2.0)
        starts = [np.array([0.0, 0.0, 0.0, 0.1, 0.3, np.arctan2(25.0, zc)])
                  for zc in np.linspace(-3.0, 3.0, 61)]
    else:
        lay = Layer(DISK, 150.0, 20, 110, 1e-5, 1e-4, hole_lo=50.0, hole_hi=55.0)
        starts = [np.array([rc, 0.0, 100.0, 0.01, 0.0, 0.05]) for rc in np.linspace(45, 60, 61)]
    seen = set()
    for margin in (0.0, 0.5):
        for p in starts:
            st0, pp, _, _, _ = O.propagate(p, None, lay, BZ, fc.kappa, check_extent=False)
            assert st0 == O.OK
            q = pp[2] if kind == BARREL else np.hypot(pp[0], pp[1])
            st, _, _, _, _ = O.propagate(p, None, lay, BZ, fc.kappa, edge_margin=margin)
            inside = lay.hole_lo + margin < q < lay.hole_hi - margin
            assert (st == O.OUT_OF_EXTENT) == inside, (q, margin, st)
            seen.add(inside)
    assert seen == {True, False}


def test_find_on_the_cms_like_geometry():
    """Small CMS-like event: stereo layers, a barrel gap and disk rings.
    The oracle's find takes each particle's own hit on the stereo layers,
    whose hits are 1.5 cm wide across the strips."""
    w = cms_like()
    ev = generate_event(w, 0, n_tracks=300)
    res = O.find_event(w.find, w.layers, ev)
    n_st = n_st_ok = 0
    for s, r in enumerate(res):
        if not r["seed_ok"]:
            continue
        tid = ev.seed_track[s]
        truth = {int(ev.layer[h]): h for h in ev.track_hits[tid]}
        for L, h in zip(r["plan"], r["hit"]):
            if w.layers[L].stereo != 0.0 and L in truth:
                n_st += 1
                n_st_ok += h == truth[L]
    assert n_st > 200
    assert n_st_ok >= 0.95 * n_st, (n_st_ok, n_st)
