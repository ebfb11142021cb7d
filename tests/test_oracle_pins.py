"""Pins of the FP64 oracle against things other than itself: Lorentz-force
integration, circle geometry, brute-force crossing search, finite
differences of an independent map, batch least squares, exhaustive search
and the statistics of the filter on simulated tracks.  CPU only."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import (BARREL, DISK, KAPPA, FindConfig, Layer, barrel_endcap, generate_event,
                   small_barrel)
from synth.workloads import barrel_layers
import helix_ref as H

BZ = 3.8


def random_states(rng, n, r_max=60.0):
    """States inside the tracker volume: position within r < r_max, pT
    0.3-10 GeV/c log-uniform, both charges, |eta| < 2.4."""
    out = []
    for _ in range(n):
        r = rng.uniform(0.0, r_max)
        a = rng.uniform(-np.pi, np.pi)
        z = rng.uniform(-100, 100)
        pt = np.exp(rng.uniform(np.log(0.3), np.log(10.0)))
        q = rng.choice([-1.0, 1.0])
        eta = rng.uniform(-2.4, 2.4)
        th = 2 * np.arctan(np.exp(-eta))
        phi = rng.uniform(-np.pi, np.pi)
        out.append(np.array([r * np.cos(a), r * np.sin(a), z, q / pt, phi, th]))
    return out


# ------------------------------------------------------------- transport

def test_transport_matches_rk4_lorentz_force():
    rng = np.random.default_rng(1)
    for p in random_states(rng, 6):
        w = KAPPA * BZ * abs(p[3])
        l = rng.uniform(0.05, 0.95) * np.pi / w
        out = O.transport(p, l, BZ, KAPPA)
        s3 = l / np.sin(p[5])
        r, u = H.rk4_track(p, s3, BZ, n_steps=4000)
        assert np.allclose(out[:3], r, atol=1e-9, rtol=0), (out[:3], r)
        assert abs(np.arctan2(u[1], u[0]) - out[4]) < 1e-10
        assert abs(np.arccos(u[2]) - out[5]) < 1e-10


def test_transport_stays_on_helix_circle_and_straight_limit():
    rng = np.random.default_rng(2)
    for p in random_states(rng, 20):
        w = -KAPPA * BZ * p[3]
        cx, cy = p[0] - np.sin(p[4]) / w, p[1] + np.cos(p[4]) / w
        for l in np.linspace(0.1, 0.99 * np.pi / abs(w), 7):
            o = O.transport(p, l, BZ, KAPPA)
            assert abs(np.hypot(o[0] - cx, o[1] - cy) - 1 / abs(w)) < 1e-10 * (1 / abs(w))
            assert abs(o[2] - (p[2] + l / np.tan(p[5]))) < 1e-11
        # B = 0: a straight line
        o = O.transport(p, 37.0, 0.0, KAPPA)
        exp = [p[0] + 37 * np.cos(p[4]), p[1] + 37 * np.sin(p[4]), p[2] + 37 / np.tan(p[5])]
        assert np.allclose(o[:3], exp, atol=1e-12)
        assert o[4] == pytest.approx(p[4], abs=1e-15)


# ------------------------------------------------------------- crossings

def test_barrel_crossing_on_surface_and_equals_brute_force():
    rng = np.random.default_rng(3)
    n_found = n_none = 0
    for p in random_states(rng, 40):
        R = rng.choice([16.0, 25.0, 43.0, 70.0])
        l = O.path_to_barrel(p, R, BZ, KAPPA)
        lb = H.brute_crossing(p, 0, R, BZ)
        if lb is None:
            assert l is None
            n_none += 1
            continue
        n_found += 1
        assert l is not None
        assert abs(l - lb) < 1e-8 * max(1.0, lb), (l, lb)
        o = O.transport(p, l, BZ, KAPPA)
        assert abs(np.hypot(o[0], o[1]) - R) < 1e-12 * R
    assert n_found > 10 and n_none > 2


def test_barrel_crossing_straight_line_limit():
    rng = np.random.default_rng(4)
    for p in random_states(rng, 20, r_max=30.0):
        R = 50.0
        a = p[0] * np.cos(p[4]) + p[1] * np.sin(p[4])
        g0 = p[0] ** 2 + p[1] ** 2 - R ** 2
        l_line = -a + np.sqrt(a * a - g0)  # textbook line-circle root (outward)
        assert O.path_to_barrel(p, R, 0.0, KAPPA) == pytest.approx(l_line, rel=1e-13)
        # continuity as the field vanishes
        assert O.path_to_barrel(p, R, 1e-7, KAPPA) == pytest.approx(l_line, rel=1e-6)


def test_disk_crossing():
    rng = np.random.default_rng(5)
    hits = 0
    for p in random_states(rng, 40):
        Z = rng.choice([-200.0, 150.0, 280.0])
        l = O.path_to_disk(p, Z, BZ, KAPPA)
        lb = H.brute_crossing(p, 1, Z, BZ)
        if lb is None:
            assert l is None
            continue
        hits += 1
        assert l == pytest.approx(lb, rel=1e-8, abs=1e-9)
        assert O.transport(p, l, BZ, KAPPA)[2] == pytest.approx(Z, abs=1e-11)
    assert hits > 5


# ------------------------------------------------- Jacobian, covariance

def _fd_jacobian(p, kind, pos, eps):
    J = np.zeros((6, 6))
    for j in range(6):
        d = np.zeros(6)
        d[j] = eps[j]
        a = H.crossing_state(p + d, kind, pos, BZ)
        b = H.crossing_state(p - d, kind, pos, BZ)
        diff = a - b
        diff[4] = np.arctan2(np.sin(diff[4]), np.cos(diff[4]))
        J[:, j] = diff / (2 * eps[j])
    return J


@pytest.mark.parametrize("kind,pos", [(0, 43.0), (0, 70.0), (1, 160.0), (1, -220.0)])
def test_surface_jacobian_matches_finite_differences(kind, pos):
    rng = np.random.default_rng(6 + kind)
    layer = Layer(kind, pos, -1e9, 1e9, 1, 1) if kind == 0 else Layer(kind, pos, 0, 1e9, 1, 1)
    checked = 0
    for p in random_states(rng, 60, r_max=12.0):
        if kind == 1 and np.sign(np.cos(p[5])) != np.sign(pos):
            continue
        st, pp, _, F, l = O.propagate(p, np.eye(6), layer, BZ, KAPPA, check_extent=False)
        if st != O.OK or H.crossing_state(p, kind, pos, BZ) is None:
            continue
        eps = np.array([1e-5, 1e-5, 1e-5, 1e-6 * abs(p[3]), 1e-7, 1e-7])
        J = _fd_jacobian(p, kind, pos, eps)
        scale = np.abs(F) + 1e-6
        assert np.all(np.abs(J - F) <= 1e-5 * scale + 1e-6), (J - F)
        checked += 1
    assert checked >= 5


def test_transported_covariance_is_rank5_psd():
    rng = np.random.default_rng(7)
    layers = [Layer(0, 34.0, -1e9, 1e9, 1, 1), Layer(1, 180.0, 0, 1e9, 1, 1)]
    n_checked = 0
    for p in random_states(rng, 40, r_max=20.0):
        A = rng.normal(size=(6, 6))
        C0 = A @ A.T * 1e-3 + np.diag([1e-3] * 6)
        for lay in layers:
            st, pp, Cp, F, l = O.propagate(p, C0, lay, BZ, KAPPA, check_extent=False)
            if st != O.OK:
                continue
            n_checked += 1
            assert np.array_equal(Cp, Cp.T)
            n = np.zeros(6)
            if lay.kind == 0:
                n[0], n[1] = pp[0], pp[1]
            else:
                n[2] = 1.0
            n /= np.linalg.norm(n)
            assert abs(n @ Cp @ n) < 1e-12 * np.trace(Cp)
            ev = np.linalg.eigvalsh(Cp)
            assert ev.min() > -1e-12 * ev.max()
            np.linalg.cholesky(Cp + np.outer(n, n))  # PD on the complement of n
    assert n_checked > 20


def test_scattering_before_or_after_update_is_identical():
    rng = np.random.default_rng(8)
    for p in random_states(rng, 20):
        A = rng.normal(size=(6, 6))
        Cm = A @ A.T * 1e-4 + 1e-5 * np.eye(6)
        hit = p[:3] + rng.normal(0, 0.01, 3)
        kind = rng.integers(0, 2)
        _, pa, Ca, ca = O.update_hit(p, O.add_ms(p, 0.001, Cm), kind, hit, 9e-6, 1e-4)
        _, pb, Cb, cb = O.update_hit(p, Cm, kind, hit, 9e-6, 1e-4)
        Cb = O.add_ms(p, 0.001, Cb)  # noise of the predicted state in both orders
        assert np.allclose(pa, pb, rtol=1e-13, atol=1e-15)
        assert np.allclose(Ca, Cb, rtol=1e-11, atol=1e-18)
        assert ca == pytest.approx(cb, rel=1e-12)


# ------------------------------------------------------------ Kalman

@pytest.mark.parametrize("joseph", [False, True])
def test_kalman_equals_batch_least_squares(joseph):
    """Static linear Gauss-Markov model (no process noise): sequential
    Kalman updates from a prior equal weighted least squares with the
    prior as a pseudo-measurement; the summed chi2 increments equal the
    least-squares objective at the minimum."""
    rng = np.random.default_rng(9)
    for _ in range(10):
        p0 = rng.normal(size=6)
        A = rng.normal(size=(6, 6))
        C0 = A @ A.T + 0.5 * np.eye(6)
        Hs, ms, Vs = [], [], []
        p, Cm, chi_sum = p0.copy(), C0.copy(), 0.0
        for k in range(7):
            Hk = rng.normal(size=(2, 6))
            B = rng.normal(size=(2, 2))
            Vk = B @ B.T + 0.1 * np.eye(2)
            mk = rng.normal(size=2) * 3
            r = mk - Hk @ p
            p, Cm, c2 = O.kf_update(p, Cm, Hk, r, Vk, joseph=joseph)
            chi_sum += c2
            Hs.append(Hk), ms.append(mk), Vs.append(Vk)
        W0 = np.linalg.inv(C0)
        Nm = W0.copy()
        b = W0 @ p0
        for Hk, mk, Vk in zip(Hs, ms, Vs):
            Wk = np.linalg.inv(Vk)
            Nm += Hk.T @ Wk @ Hk
            b += Hk.T @ Wk @ mk
        p_ls = np.linalg.solve(Nm, b)
        C_ls = np.linalg.inv(Nm)
        obj = (p_ls - p0) @ W0 @ (p_ls - p0) + sum(
            (mk - Hk @ p_ls) @ np.linalg.inv(Vk) @ (mk - Hk @ p_ls) for Hk, mk, Vk in zip(Hs, ms, Vs))
        assert np.allclose(p, p_ls, rtol=1e-9, atol=1e-10)
        assert np.allclose(Cm, C_ls, rtol=1e-8, atol=1e-12)
        assert chi_sum == pytest.approx(obj, rel=1e-9)


def test_measurement_frame_barrel_and_disk():
    p = np.array([30.0, 40.0, 10.0, 0.5, 0.3, 1.0])  # r = 50
    ok, r, Hm = O.measure(p, 0, np.array([30.0 - 0.4 * 0.01, 40.0 + 0.3 * 0.01, 10.02]))
    assert ok
    # t = (-0.8, 0.6); dx = (-0.004, 0.003): u = 0.0032 + 0.0018
    assert r == pytest.approx([0.005, 0.02], abs=1e-12)
    assert Hm[0, :2] == pytest.approx([-0.8, 0.6]) and Hm[1, 2] == 1.0
    ok, _, _ = O.measure(p, 0, np.array([-30.0, -40.0, 10.0]))  # other half
    assert not ok
    ok, r, Hm = O.measure(p, 1, np.array([30.0 + 0.6 * 0.05, 40.0 + 0.8 * 0.05, 10.0]))
    assert ok and r == pytest.approx([0.0, 0.05], abs=1e-12)


# ------------------------------------------------------------- seeding

def test_seed_of_noise_free_triplet_is_exact():
    fc = FindConfig(ms_sigma=0.0)
    layers = barrel_layers()
    rng = np.random.default_rng(11)
    n_ok = 0
    for p in random_states(rng, 30, r_max=0.01):
        p[2] = rng.uniform(-5, 5)
        p[5] = 2 * np.arctan(np.exp(-rng.uniform(-0.8, 0.8)))
        if abs(p[3]) > 2.0:
            continue
        states = []
        cur = p
        for R in (4.0, 7.0, 11.0):
            s = H.crossing_state(cur, 0, R, BZ)
            states.append(s)
            cur = s
        h = np.array([s[:3] for s in states]).ravel()
        out = O.seed(fc, layers, h, [9e-6, 1e-4] * 3, [0, 1, 2])
        assert out["ok"]
        truth = states[2]
        d = out["par"] - truth
        d[4] = np.arctan2(np.sin(d[4]), np.cos(d[4]))
        assert np.all(np.abs(d) <= 1e-9 * np.maximum(1.0, np.abs(truth))), d
        assert list(out["plan"]) == [3, 4, 5, 6, 7, 8, 9]
        n_ok += 1
    assert n_ok > 10


# -------------------------------------------------------------- finding

def test_find_recovers_truth_on_small_barrel_event():
    w = small_barrel()
    ev = generate_event(w, 0)
    res = O.find_event(w.find, w.layers, ev)
    assert len(res) == 200
    for s, r in enumerate(res):
        truth = ev.track_hits[ev.seed_track[s]][3:]
        assert r["seed_ok"] and r["n_hits"] == 10
        assert list(r["hit"]) == list(truth)


def _exhaustive_best(fc, layers, ev, seed_hits, tol_unused=None):
    """All extension paths by recursion, using only the oracle's single-state
    primitives; best by (more hits, smaller chi2)."""
    h = np.array([[ev.x[i], ev.y[i], ev.z[i]] for i in seed_hits], float).ravel()
    hv = np.array([[ev.var_u[i], ev.var_v[i]] for i in seed_hits], float).ravel()
    hl = [int(ev.layer[i]) for i in seed_hits]
    sd = O.seed(fc, layers, h, hv, hl)
    plan = sd["plan"]
    by_layer = {L: np.nonzero(ev.layer == L)[0] for L in set(plan.tolist())}
    leaves = []

    def rec(step, p, Cm, n_hits, n_miss, chi, hist):
        if step == len(plan):
            leaves.append((n_hits, chi, hist))
            return
        lay = layers[plan[step]]
        st, pp, Cp, _, _ = O.propagate(p, Cm, lay, fc.bz, fc.kappa, fc.l_min, fc.edge_margin, True)
        if st != O.OK:
            rec(step + 1, p, Cm, n_hits, n_miss, chi, hist + [O.HIT_SKIP])
            return
        Cp = O.add_ms(pp, fc.ms_sigma, Cp)
        any_ext = False
        for i in by_layer[plan[step]]:
            hit = np.array([ev.x[i], ev.y[i], ev.z[i]], float)
            c2 = O.chi2(pp, Cp, lay.kind, hit, float(ev.var_u[i]), float(ev.var_v[i]))
            if c2 is not None and c2 < fc.chi2_cut:
                any_ext = True
                _, pu, Cu, _ = O.update_hit(pp, Cp, lay.kind, hit, float(ev.var_u[i]),
                                            float(ev.var_v[i]))
                rec(step + 1, pu, Cu, n_hits + 1, n_miss, chi + c2, hist + [int(i)])
        if n_miss < fc.max_holes:
            any_ext = True
            rec(step + 1, pp, Cp, n_hits, n_miss + 1, chi, hist + [O.HIT_MISS])
        if not any_ext:
            leaves.append((n_hits, chi, hist + [O.HIT_NONE] * (len(plan) - step)))

    rec(0, sd["par"], sd["cov"], 3, 0, 0.0, [])
    leaves.sort(key=lambda t: (-t[0], t[1]))
    return plan, leaves


def test_clone_engine_with_unbounded_budget_equals_exhaustive_search():
    """Tiny events (2 tracks plus noise, barrel + disks): with a candidate
    budget larger than the number of paths, the clone engine's best track
    is the best complete path of a recursive enumeration."""
    w = barrel_endcap()
    fc = FindConfig(n_cand=400, max_holes=2)
    n_cases = 0
    for e in range(6):
        ev = generate_event(w, 1000 + e, n_tracks=2)
        if ev.seeds.shape[0] == 0:
            continue
        # add dense noise close to the tracks: copies of true hits shifted by
        # a few hit sigmas, so that several hits compete on each layer
        rng = np.random.default_rng(e)
        true_idx = np.nonzero(ev.track >= 0)[0]
        extra = rng.choice(true_idx, size=min(12, true_idx.size), replace=False)
        from synth.events import Event
        sh = rng.normal(0, 0.02, (extra.size, 3)).astype(np.float32)
        ev2 = Event(np.concatenate([ev.x, ev.x[extra] + sh[:, 0]]),
                    np.concatenate([ev.y, ev.y[extra] + sh[:, 1]]),
                    np.concatenate([ev.z, ev.z[extra] + sh[:, 2]]),
                    np.concatenate([ev.var_u, ev.var_u[extra]]),
                    np.concatenate([ev.var_v, ev.var_v[extra]]),
                    np.concatenate([ev.layer, ev.layer[extra]]),
                    np.concatenate([ev.track, np.full(extra.size, -1, np.int32)]),
                    ev.seeds, ev.seed_track, None, ev.track_hits)
        res = O.find_event(fc, w.layers, ev2)
        for s in range(ev2.seeds.shape[0]):
            plan, leaves = _exhaustive_best(fc, w.layers, ev2, ev2.seeds[s])
            assert list(res[s]["plan"]) == list(plan)
            best = leaves[0]
            assert res[s]["n_hits"] == best[0]
            assert res[s]["chi2"] == pytest.approx(best[1], rel=1e-12, abs=1e-12)
            assert list(res[s]["hit"]) == best[2]
            n_cases += 1
    assert n_cases >= 6


def test_candidate_budget_one_is_greedy():
    """With one candidate kept, each layer takes the single best extension
    of the single candidate: best hit if any, else miss/skip."""
    w = barrel_endcap()
    fc = FindConfig(n_cand=1)
    ev = generate_event(w, 7, n_tracks=50)
    res = O.find_event(fc, w.layers, ev)
    for s in range(min(20, ev.seeds.shape[0])):
        sh = ev.seeds[s]
        plan, leaves = _exhaustive_best(FindConfig(n_cand=1), w.layers, ev, sh)
        # follow the greedy path through the enumeration: at each step the
        # chosen extension has the most hits, then the least chi2
        hist = list(res[s]["hit"])
        assert len(hist) == len(plan)
        assert any(l[2] == hist for l in leaves)


# ---------------------------------------------------------- statistics

def test_fit_chi2_and_pulls_on_simulated_tracks():
    """The paper's own validation criterion (Introduction): the chi2
    distribution and the pulls of the track parameters.  Fitting each
    simulated track through its true hits must give a per-hit chi2 mean of
    2 (2 dof) and pulls of mean 0 and width 1."""
    w = barrel_endcap()
    fc = w.find
    ev = generate_event(w, 3, n_tracks=600)
    chis, pulls = [], []
    for t, hits in enumerate(ev.track_hits):
        if hits.shape[0] < 8:
            continue
        h = np.array([[ev.x[i], ev.y[i], ev.z[i]] for i in hits[:3]], float).ravel()
        hv = np.array([[ev.var_u[i], ev.var_v[i]] for i in hits[:3]], float).ravel()
        sd = O.seed(fc, w.layers, h, hv, [int(ev.layer[i]) for i in hits[:3]])
        if not sd["ok"]:
            continue
        rest = hits[3:]
        kinds = [w.layers[ev.layer[i]].kind for i in rest]
        pos = [w.layers[ev.layer[i]].pos for i in rest]
        hh = np.array([[ev.x[i], ev.y[i], ev.z[i]] for i in rest], float)
        rc, p, Cm, c2 = O.fit_track(fc, sd["par"], sd["cov"], kinds, pos, hh,
                                    ev.var_u[rest].astype(float), ev.var_v[rest].astype(float))
        assert rc == 0
        chis.append(c2 / rest.shape[0])
        truth = ev.truth_state[rest[-1]]
        d = p - truth
        d[4] = np.arctan2(np.sin(d[4]), np.cos(d[4]))
        pulls.append(d[3:] / np.sqrt(np.diag(Cm)[3:]))
    chis = np.array(chis)
    pulls = np.array(pulls)
    assert chis.size > 300
    assert abs(chis.mean() - 2.0) < 0.12, chis.mean()
    for k in range(3):
        assert abs(pulls[:, k].mean()) < 0.12, (k, pulls[:, k].mean())
        assert abs(pulls[:, k].std() - 1.0) < 0.12, (k, pulls[:, k].std())
