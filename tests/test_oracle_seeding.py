"""Pins of the oracle's combinatorial triplet seeding against things other
than itself: the known helix of exact crossing points (pT, d0, z0 from the
generating state by circle geometry and dense sampling), the direction of
every cut, and the true triplets of simulated events.  CPU only."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import FindConfig, SeedingConfig, barrel_endcap, generate_event, small_barrel
import helix_ref as H

BZ = 3.8
RADII = (4.0, 7.0, 11.0)


def vertex_state(rng, pt_lo=0.3):
    pt = np.exp(rng.uniform(np.log(pt_lo), np.log(10.0)))
    q = rng.choice([-1.0, 1.0])
    th = 2 * np.arctan(np.exp(-rng.uniform(-2.4, 2.4)))
    return np.array([rng.normal(0, 0.02), rng.normal(0, 0.02), rng.uniform(-10, 10), q / pt,
                     rng.uniform(-np.pi, np.pi), th]), pt


def exact_hits(p):
    out, cur = [], p
    for R in RADII:
        cur = H.crossing_state(cur, 0, R, BZ)
        assert cur is not None
        out.append(cur)
    return out


def truth_d0_z0(p):
    """Distance of the true circle from the beam line (circle geometry) and
    z at its point of closest approach (dense sampling of the helix)."""
    w = -O.make_cfg(FindConfig()).kappa * BZ * p[3]
    cx, cy = p[0] - np.sin(p[4]) / w, p[1] + np.cos(p[4]) / w
    d0 = abs(np.hypot(cx, cy) - 1 / abs(w))
    ls = np.linspace(-2.0, 2.0, 400001)
    pts = np.array([H.centre_form(p, l, BZ) for l in ls[::1000]])
    i = np.argmin(np.hypot(pts[:, 0], pts[:, 1]))
    fine = np.linspace(ls[::1000][max(i - 1, 0)], ls[::1000][min(i + 1, len(pts) - 1)], 20001)
    fp = np.array([H.centre_form(p, l, BZ) for l in fine])
    j = np.argmin(np.hypot(fp[:, 0], fp[:, 1]))
    return d0, fp[j, 2]


def test_cut_variables_of_exact_points_are_the_helix_parameters():
    fc, sc = FindConfig(), SeedingConfig()
    rng = np.random.default_rng(41)
    for _ in range(25):
        p, pt = vertex_state(rng)
        hits = exact_hits(p)
        ok, margin, v = O.triplet_params(fc, sc, *[h[:3] for h in hits])
        d0, z0 = truth_d0_z0(p)
        assert v[0] == pytest.approx(pt, rel=1e-9)
        assert v[1] == pytest.approx(d0, abs=1e-9)
        assert abs(v[2]) < 1e-9                      # the points lie on one s-z line
        assert v[3] == pytest.approx(z0, abs=2e-4)   # dense sampling: 1e-5 cm steps
        assert 0 < v[4] < v[5] < np.pi and v[6] < np.pi
        assert ok == (pt >= sc.pt_min and d0 <= sc.d0_max and abs(z0) <= sc.z0_max)


@pytest.mark.parametrize("cut", ["pt_min", "d0_max", "z0_max", "dz_max"])
def test_each_cut_passes_just_inside_and_fails_just_outside(cut):
    fc = FindConfig()
    rng = np.random.default_rng(42)
    p, _ = vertex_state(rng, pt_lo=1.0)
    hits = [h[:3].copy() for h in exact_hits(p)]
    if cut == "dz_max":
        hits[1][2] += 0.05  # a middle hit off the s-z line
    ok, _, v = O.triplet_params(fc, SeedingConfig(), *hits)
    val = {"pt_min": v[0], "d0_max": v[1], "z0_max": abs(v[3]), "dz_max": abs(v[2])}[cut]
    lo = SeedingConfig(**{cut: val * (1 + 1e-6)})
    hi = SeedingConfig(**{cut: val * (1 - 1e-6)})
    inside, outside = (hi, lo) if cut == "pt_min" else (lo, hi)
    assert O.triplet_params(fc, inside, *hits)[0]
    assert not O.triplet_params(fc, outside, *hits)[0]


def test_order_along_the_track_is_required():
    """Swapping the middle and outer hits breaks the order along the
    circle; reversing the direction (a and c swapped) puts the beam line
    behind the first hit."""
    fc, sc = FindConfig(), SeedingConfig()
    rng = np.random.default_rng(43)
    p, _ = vertex_state(rng, pt_lo=1.0)
    a, b, c = [h[:3] for h in exact_hits(p)]
    assert O.triplet_params(fc, sc, a, b, c)[0]
    assert not O.triplet_params(fc, sc, a, c, b)[0]
    assert not O.triplet_params(fc, sc, c, b, a)[0]


def test_every_true_triplet_passes_on_simulated_events():
    """Small barrel (no material) and a realistic event (scattering,
    inefficiency, noise): the first three layers' hits of every track that
    has one on each of them pass; the accepted set is those plus fakes."""
    for w, nt in ((small_barrel(), 200), (barrel_endcap(), 150)):
        ev = generate_event(w, 3, n_tracks=nt)
        sc = SeedingConfig()
        trip, frag, _ = O.triplet_seeds(w.find, sc, ev)
        found = {tuple(t) for t in trip}
        n_true = 0
        for t, hits in enumerate(ev.track_hits):
            lay = ev.layer[hits]
            if not (len(hits) >= 3 and list(lay[:3]) == [0, 1, 2]):
                continue
            p0 = ev.truth_state[hits[0]]
            if 1 / abs(p0[3]) < sc.pt_min * 1.05:
                continue
            n_true += 1
            assert tuple(hits[:3]) in found, (t, hits[:3])
        assert n_true > 0.8 * nt
        assert len(found) >= n_true
