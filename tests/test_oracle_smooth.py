"""Pins of the oracle's Rauch-Tung-Striebel smoother of found tracks against
things other than itself: the find's own final state, the helix (without
scattering the smoothed states of one track lie on one helix), the backward
filter (a different algorithm reaching the same full-information estimate),
and the pulls against the simulated truth.  CPU only."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import FindConfig, barrel_endcap, generate_event, small_barrel
import parity as PT


def wrap(a):
    return np.arctan2(np.sin(a), np.cos(a))


def seed_state(w, ev, sh, fc=None):
    fc = fc or w.find
    h = np.array([[ev.x[i], ev.y[i], ev.z[i]] for i in sh], float).ravel()
    hv = np.array([[ev.var_u[i], ev.var_v[i]] for i in sh], float).ravel()
    return O.seed(fc, w.layers, h, hv, [int(ev.layer[i]) for i in sh])


def pos_dev(d, ref, C):
    """Deviation d of a barrel state split into its radial part (the pinned
    direction) and its azimuthal part in units of its sigma."""
    r = np.hypot(ref[0], ref[1])
    rh = np.array([ref[0], ref[1]]) / r
    th = np.array([-ref[1], ref[0]]) / r
    return abs(rh @ d[:2]), abs(th @ d[:2]) / np.sqrt(th @ C[:2, :2] @ th)


def smooth(w, ev, s, trk, fc=None):
    fc = fc or w.find
    sh = ev.seeds[s]
    sd = seed_state(w, ev, sh, fc)
    return O.smooth_track(fc, w.layers, ev, int(ev.layer[sh[2]]), sd["par"], sd["cov"], trk)


@pytest.mark.parametrize("wname", ["small_barrel", "barrel_endcap"])
def test_smoother_ends_on_the_found_state(wname):
    """The forward pass is the find's filter along the track: the last
    smoothed state is the find's final state, bit for bit, and there is one
    surface per crossed plan layer plus the seed's."""
    w = small_barrel() if wname == "small_barrel" else barrel_endcap()
    ev = generate_event(w, 1, n_tracks=200)
    res = O.find_event(w.find, w.layers, ev)
    n_ok = 0
    for s, r in enumerate(res):
        if not r["seed_ok"]:
            assert smooth(w, ev, s, r)[0] == 0
            continue
        n, lay, par, cov = smooth(w, ev, s, r)
        crossed = [L for L, h in zip(r["plan"], r["hit"]) if h >= O.HIT_MISS]
        assert n == 1 + len(crossed)
        assert list(lay[1:]) == crossed
        assert np.array_equal(par[-1], r["par"]) and np.array_equal(cov[-1], r["cov"])
        n_ok += 1
    assert n_ok > 150


def test_smoothed_states_lie_on_one_helix_without_scattering():
    """With no scattering the smoothed states of a track are one helix:
    each, carried to the next surface, is the next one, up to the
    linearisation of the transport at the filtered rather than the smoothed
    states (over all 200 tracks: worst 0.14 sigma and 5.2e-3 in correlation
    units, median 1.4e-4; a sign or transpose error gives order one)."""
    w = small_barrel()
    ev = generate_event(w, 0)
    res = O.find_event(w.find, w.layers, ev)
    worst = 0.0
    for s in range(0, 200, 5):
        n, lay, par, cov = smooth(w, ev, s, res[s])
        assert n == 8
        for k in range(n - 1):
            st, q, Q, _, _ = O.propagate(par[k], cov[k], w.layers[lay[k + 1]], w.find.bz,
                                         w.find.kappa, check_extent=False)
            assert st == O.OK
            d = q - par[k + 1]
            d[4] = wrap(d[4])
            sig = np.sqrt(np.maximum(np.diag(cov[k + 1]), 1e-30))
            dr, dt = pos_dev(d, par[k + 1], cov[k + 1])
            # Kalman and smoother corrections are linear: a shift dt along
            # the tangent plane leaves a cylinder of radius R by dt^2 / 2R
            # (the find's own filtered states sit up to 3e-5 cm off their
            # cylinders after a 300 um correction); 2e-4 cm is 1/15 of the
            # hit resolution
            assert dr < 2e-4, d
            worst = max(worst, dt, float(np.max(np.abs(d[2:]) / sig[2:])))
            assert PT.cov_err(Q, cov[k + 1]) < 1e-2
    assert worst < 0.25, worst


def test_smoother_agrees_with_the_backward_fit_without_scattering():
    """The smoothed state on the seed's third layer and the backward fit's
    state on its first layer, carried there, are the same full-information
    estimate, up to the linearisation of two different filters (over all
    200 tracks: worst 0.15 sigma, 5.4e-3 in correlation units).  With a
    seed prior that keeps its extent along the first layer's normal the
    two differed by up to 1.85 sigma: a state on a surface has no freedom
    there."""
    w = small_barrel()
    ev = generate_event(w, 0)
    res = O.find_event(w.find, w.layers, ev)
    for s in range(0, 200, 9):
        n, lay, par, cov = smooth(w, ev, s, res[s])
        st, pb, Cb, _, _ = O.backward_fit(w.find, w.layers, ev, ev.seeds[s], res[s])
        assert st == 1
        stp, q, Q, _, _ = O.propagate(pb, Cb, w.layers[lay[0]], w.find.bz, w.find.kappa,
                                      check_extent=False)
        assert stp == O.OK
        d = q - par[0]
        d[4] = wrap(d[4])
        sig = np.sqrt(np.maximum(np.diag(cov[0]), 1e-30))
        dr, dt = pos_dev(d, par[0], cov[0])
        assert dr < 2e-4 and dt < 0.25, (d, dt)
        assert np.all(np.abs(d[2:]) < 0.25 * sig[2:]), (d, sig)
        assert PT.cov_err(Q, cov[0]) < 1e-2


def test_smoothed_pulls_on_simulated_tracks():
    """With scattering: on every surface with a hit of the track's own
    particle, the smoothed q/pT, phi, theta and z (barrel) have pulls of
    mean 0 and width 1 against the simulated state after that layer."""
    w = barrel_endcap()
    ev = generate_event(w, 4, n_tracks=400)
    res = O.find_event(w.find, w.layers, ev)
    pulls = []
    for s, r in enumerate(res):
        if not r["seed_ok"]:
            continue
        tid = ev.seed_track[s]
        hits = [h for h in r["hit"] if h >= 0]
        if any(ev.track[h] != tid for h in hits):
            continue  # a noise or foreign hit: the truth is not this model's
        n, lay, par, cov = smooth(w, ev, s, r)
        assert n > 0
        k = 1
        for L, h in zip(r["plan"], r["hit"]):
            if h < O.HIT_MISS:
                continue
            if h >= 0:
                t = ev.truth_state[h]
                d = par[k] - t
                d[4] = wrap(d[4])
                sg = np.sqrt(np.diag(cov[k]))
                row = [d[3] / sg[3], d[4] / sg[4], d[5] / sg[5]]
                row.append(d[2] / sg[2] if w.layers[L].kind == 0 else np.nan)
                pulls.append(row)
            k += 1
    P = np.array(pulls)
    assert P.shape[0] > 2000
    for j in range(4):
        v = P[:, j][np.isfinite(P[:, j])]
        assert abs(v.mean()) < 0.1, (j, v.mean())
        assert abs(v.std() - 1.0) < 0.1, (j, v.std())
