"""Pins of the oracle's seed cleaning: a hand-worked example of the rule
(shared hit, parameter tolerances, ranking), invariance under reordering,
and on a dense simulated event seeded from every triplet, no particle left
without a seed.  CPU only."""
import numpy as np

from oracle import oracle as O
from synth import CleaningConfig, SeedingConfig, barrel_endcap, generate_event


def state(ipt, phi, eta):
    return [0.0, 0.0, 0.0, ipt, phi, 2 * np.arctan(np.exp(-eta))]


def test_hand_worked_example():
    cc = CleaningConfig()
    trip = [[1, 2, 3],      # 0: best chi2 of the particle
            [1, 2, 4],      # 1: shares 1, 2 with 0, close: removed
            [1, 5, 6],      # 2: shares 1 with 0 but q/pT 20% off: kept
            [7, 8, 3],      # 3: shares 3 with 0, eta 0.03 off: kept
            [9, 10, 4],     # 4: shares 4 with 1 (removed itself) and is close to it: removed
            [11, 12, 13],   # 5: shares nothing: kept
            [11, 12, 14]]   # 6: same chi2 as 5, close, larger triplet: removed
    par = [state(1.0, 0.5, 0.3), state(1.05, 0.51, 0.31), state(1.2, 0.5, 0.3),
           state(1.0, 0.5, 0.33), state(1.05, 0.515, 0.31), state(-0.5, 1.0, -1.0),
           state(-0.5, 1.0, -1.0)]
    chi2 = [0.5, 1.0, 0.1, 0.2, 2.0, 0.7, 0.7]
    ok = [1] * 7
    keep, frag = O.clean_seeds(trip, ok, par, chi2, cc.tol_ipt, cc.tol_eta, cc.tol_phi)
    assert list(keep) == [True, False, True, True, False, True, False]
    assert frag[5] and frag[6]      # the chi2 tie
    assert not frag[0] and not frag[1]
    # a failed fit is dropped and removes nothing
    ok2 = [0] + [1] * 6
    keep2, _ = O.clean_seeds(trip, ok2, par, chi2, cc.tol_ipt, cc.tol_eta, cc.tol_phi)
    assert list(keep2) == [False, True, True, True, False, True, False]


def test_flags_do_not_depend_on_seed_order():
    rng = np.random.default_rng(61)
    n = 80
    trip = np.sort(rng.integers(0, 60, (n, 3)), axis=1)
    par = [state(rng.choice([0.5, 0.52, 1.0]), rng.choice([0.1, 0.11]), rng.choice([0.2, 0.21]))
           for _ in range(n)]
    chi2 = rng.integers(0, 6, n).astype(float)
    ok = rng.random(n) > 0.1
    cc = CleaningConfig()
    keep, _ = O.clean_seeds(trip, ok, par, chi2, cc.tol_ipt, cc.tol_eta, cc.tol_phi)
    perm = rng.permutation(n)
    keep2, _ = O.clean_seeds(trip[perm], ok[perm], [par[i] for i in perm], chi2[perm],
                             cc.tol_ipt, cc.tol_eta, cc.tol_phi)
    assert np.array_equal(keep2, keep[perm])


def dense_event(w, e):
    """300 tracks within 0.15 rad of azimuth: the local hit density of
    ~12,000 tracks over the full circle."""
    return generate_event(w, e, n_tracks=300, phi_range=(0.0, 0.15))


def test_no_particle_loses_all_its_seeds():
    """Dense jet-like event seeded from every triplet: cleaning removes a
    share of the seeds, and every particle that had a seed made of its own
    first three hits keeps a seed sharing at least two of them."""
    w = barrel_endcap()
    ev = dense_event(w, 6)
    sc, cc = SeedingConfig(), CleaningConfig()
    trip, _, _ = O.triplet_seeds(w.find, sc, ev)
    fits = [O.seed(w.find, w.layers, np.array([[ev.x[i], ev.y[i], ev.z[i]] for i in t]).ravel(),
                   np.array([[ev.var_u[i], ev.var_v[i]] for i in t]).ravel(),
                   [int(ev.layer[i]) for i in t]) for t in trip]
    keep, _ = O.clean_seeds(trip, [f["ok"] for f in fits], [f["par"] for f in fits],
                            [f["chi2"] for f in fits], cc.tol_ipt, cc.tol_eta, cc.tol_phi)
    assert keep.sum() < 0.95 * len(trip)
    kept = [set(t) for t, k in zip(trip, keep) if k]
    by_hit = {}
    for s in kept:
        for h in s:
            by_hit.setdefault(h, []).append(s)
    n_part = 0
    for t, hits in enumerate(ev.track_hits):
        first = tuple(hits[:3])
        if len(hits) < 3 or first not in {tuple(x) for x in trip[trip[:, 0] == hits[0]]}:
            continue
        n_part += 1
        assert any(len(s & set(first)) >= 2 for s in by_hit.get(hits[0], []) +
                   by_hit.get(hits[1], []) + by_hit.get(hits[2], [])), first
    assert n_part > 200
