"""Pins of the oracle's propagation in a parameterised field (Section 2.1: a
constant or a parameterised field, selectable per propagation): in a uniform
field the Runge-Kutta crossing is the closed-form one; the steps converge at
fourth order; the mean-curvature Jacobian against finite differences of the
stepped transport; and on simulated events in a solenoid-like field the
find and the backward fit have unbiased pulls, where assuming a uniform
field does not.  CPU only."""
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle as O
from synth import (BARREL, DISK, KAPPA, FieldMap, Layer, barrel_endcap_field, generate_event,
                   solenoid_field)

BZ = 3.8
LAYERS = (Layer(BARREL, 52.0, -300, 300, 1e-5, 1e-4), Layer(DISK, 200.0, 0, 300, 1e-5, 1e-4),
          Layer(DISK, -150.0, 0, 300, 1e-5, 1e-4))


def states(rng, n=20):
    out = []
    for _ in range(n):
        a = rng.uniform(-np.pi, np.pi)
        r = rng.uniform(3.0, 15.0)
        pt = rng.uniform(1.0, 5.0)
        th = rng.choice([rng.uniform(0.5, 1.2), rng.uniform(2.0, 2.6)])
        out.append(np.array([r * np.cos(a), r * np.sin(a), rng.uniform(-10, 10),
                             rng.choice([-1, 1]) / pt, a + rng.uniform(-0.3, 0.3), th]))
    return out


def crossings(field, ps):
    for p in ps:
        for L in LAYERS:
            yield p, L, O.propagate(p, np.eye(6), L, BZ, KAPPA, check_extent=False, field=field)


def test_uniform_field_steps_match_the_closed_form():
    """With c = 0 the stepped transport is the exact helix: to RK4's
    truncation (1e-9 cm at 0.5 cm steps, 1e-6 cm at 5 cm) and the rounding
    of the Newton end."""
    rng = np.random.default_rng(61)
    ps = states(rng)
    n = 0
    for h, tol in ((0.5, 1e-6), (5.0, 1e-5)):
        for p, L, (st, q, Cq, F, l) in crossings(FieldMap(b0=BZ, h_max=h), ps):
            # the field's coefficients reach the oracle at FP32, as the library's do
            st0, q0, C0, F0, l0 = O.propagate(p, np.eye(6), L, float(np.float32(BZ)), KAPPA,
                                              check_extent=False)
            assert st == st0
            if st != O.OK:
                continue
            n += 1
            d = q - q0
            d[4] = np.arctan2(np.sin(d[4]), np.cos(d[4]))
            assert np.abs(d[:3]).max() < tol and abs(d[4]) < tol / 10 and abs(l - l0) < tol
            assert np.abs(F - F0).max() < 100 * tol * max(1.0, np.abs(F0).max())
    assert n > 40


def test_steps_converge_at_fourth_order():
    """In the solenoid-like field, halving the step divides the error of the
    crossing point by ~16."""
    rng = np.random.default_rng(62)
    f = solenoid_field()
    n = 0
    for p in states(rng, 8):
        for L in LAYERS:
            ref = O.propagate(p, None, L, BZ, KAPPA, check_extent=False,
                              field=replace(f, h_max=0.05))
            if ref[0] != O.OK:
                continue
            e = [np.abs(O.propagate(p, None, L, BZ, KAPPA, check_extent=False,
                                    field=replace(f, h_max=h))[1][:3] - ref[1][:3]).max()
                 for h in (20.0, 10.0, 5.0)]
            if e[1] < 1e-8:     # already at rounding level
                continue
            n += 1
            assert 8.0 < e[0] / e[1] < 32.0 and e[1] > e[2], e
    assert n >= 8


def layer_steps(rng, n):
    """States one layer before the LAYERS (9 cm inside the cylinder, 20 cm
    before each disk), heading to them: the find's propagations."""
    out = []
    for _ in range(n):
        a = rng.uniform(-np.pi, np.pi)
        pt = rng.uniform(1.0, 5.0)
        q = rng.choice([-1, 1]) / pt
        out.append((np.array([43.0 * np.cos(a), 43.0 * np.sin(a), rng.uniform(-60, 60), q,
                              a + rng.uniform(-0.2, 0.2), rng.uniform(0.8, 2.3)]), LAYERS[0]))
        r = rng.uniform(40.0, 80.0)
        out.append((np.array([r * np.cos(a), r * np.sin(a), 180.0, q, a + rng.uniform(-0.2, 0.2),
                              rng.uniform(0.25, 0.5)]), LAYERS[1]))
        out.append((np.array([r * np.cos(a), r * np.sin(a), -130.0, q, a + rng.uniform(-0.2, 0.2),
                              np.pi - rng.uniform(0.25, 0.5)]), LAYERS[2]))
    return out


def test_mean_curvature_jacobian_against_finite_differences():
    """The Jacobian is that of the helix with the path's mean curvature,
    made surface-constrained; it misses the field's change along the varied
    paths.  For layer-to-layer steps in the solenoid-like field (where the
    field falls fastest, beyond the barrel's ends) that stays below 0.2% of
    the largest element; a sign or index error is of order one."""
    rng = np.random.default_rng(63)
    f = solenoid_field()
    worst = 0.0
    n = 0
    for p, L in layer_steps(rng, 8):
        st, q, _, F, _ = O.propagate(p, np.eye(6), L, BZ, KAPPA, check_extent=False, field=f)
        if st != O.OK:
            continue
        Fn = np.zeros((6, 6))
        for j in range(6):
            e = 1e-6 * max(1.0, abs(p[j]))
            dp = np.zeros(6)
            dp[j] = e
            qa = O.propagate(p + dp, None, L, BZ, KAPPA, check_extent=False, field=f)[1]
            qb = O.propagate(p - dp, None, L, BZ, KAPPA, check_extent=False, field=f)[1]
            d = qa - qb
            d[4] = np.arctan2(np.sin(d[4]), np.cos(d[4]))
            Fn[:, j] = d / (2 * e)
        worst = max(worst, np.abs(F - Fn).max() / np.abs(F).max())
        n += 1
    # measured: 5.0e-4
    assert n > 20 and worst < 2e-3, worst


@pytest.fixture(scope="module")
def field_event():
    w = barrel_endcap_field()
    return w, generate_event(w, 0, n_tracks=300)


def abs_ipt_pulls(w, ev, field):
    res = O.find_event(w.find, w.layers, ev, field=field)
    fwd, bwd = [], []
    for s, r in enumerate(res):
        if not r["seed_ok"]:
            continue
        if len(r["hit"]) and r["hit"][-1] >= 0:
            t = ev.truth_state[r["hit"][-1]]
            fwd.append((abs(r["par"][3]) - abs(t[3])) / np.sqrt(r["cov"][3, 3]))
        st, p, Cm, _, _ = O.backward_fit(w.find, w.layers, ev, ev.seeds[s], r, field=field)
        if st == 1:
            t0 = ev.track_init[ev.seed_track[s]]
            bwd.append((abs(p[3]) - abs(t0[3])) / np.sqrt(Cm[3, 3]))
    return np.array(fwd), np.array(bwd), sum(r["n_hits"] for r in res)


def test_pulls_in_the_solenoid_like_field(field_event):
    """300 tracks of the realistic recipe simulated in the solenoid-like
    field (the generator's own fine Runge-Kutta steps): the find's |q/pT|
    at the last hit and the backward fit's at the vertex have pulls of mean
    ~0 and width ~1; assuming the uniform 3.8 T instead gives pulls of width
    above 2 and loses hits."""
    w, ev = field_event
    fwd, bwd, hits = abs_ipt_pulls(w, ev, w.field)
    assert len(fwd) > 200 and len(bwd) > 250
    assert abs(fwd.mean()) < 0.2 and 0.85 < fwd.std() < 1.15, (fwd.mean(), fwd.std())
    assert abs(bwd.mean()) < 0.2 and 0.85 < bwd.std() < 1.15, (bwd.mean(), bwd.std())
    fwd_u, _, hits_u = abs_ipt_pulls(w, ev, None)
    assert fwd_u.std() > 2.0 and hits_u < 0.97 * hits


def test_barrel_crossing_lies_on_the_cylinder_for_any_step():
    """The last step's length is solved to convergence: whatever the step
    size, from the smallest the library accepts (0.01 cm) to the largest
    (100 cm, where one Runge-Kutta step spans the whole path and its
    secant guess is far off), the end point of the stepped path lies on
    r = R to rounding."""
    rng = np.random.default_rng(64)
    f = solenoid_field()
    L = Layer(BARREL, 70.0, -300, 300, 1e-5, 1e-4)
    n = 0
    for p in states(rng, 10):
        for h in (0.01, 0.5, 20.0, 100.0):
            st, q, _, _, l = O.propagate(p, None, L, BZ, KAPPA, check_extent=False,
                                         field=replace(f, h_max=h))
            assert st == O.OK, (p, h)
            assert abs(np.hypot(q[0], q[1]) - 70.0) < 1e-10 * 70.0, (h, np.hypot(q[0], q[1]))
            n += 1
    assert n == 40


def test_smallest_step_reaches_a_crossing_sixty_cm_away():
    """At the smallest step the library accepts (0.01 cm) the search runs as
    far as at any other step (1000 cm of path, half a turn): a barrel
    crossing ~66 cm away (6,600 steps) and a disk 150 cm away are found;
    in a uniform field they equal the closed-form crossings, and in the
    solenoid-like field they equal the 0.25 cm-step crossings to the
    Runge-Kutta truncation."""
    rng = np.random.default_rng(65)
    f = solenoid_field()
    barrel = Layer(BARREL, 70.0, -300, 300, 1e-5, 1e-4)
    disk = Layer(DISK, 150.0, 0, 300, 1e-5, 1e-4)
    n = 0
    for _ in range(6):
        a = rng.uniform(-np.pi, np.pi)
        pt = rng.uniform(2.0, 8.0)
        p = np.array([4.0 * np.cos(a), 4.0 * np.sin(a), rng.uniform(-5, 5),
                      rng.choice([-1, 1]) / pt, a + rng.uniform(-0.1, 0.1), 0.9])
        for L in (barrel, disk):
            st0, q0, _, _, l0 = O.propagate(p, None, L, float(np.float32(BZ)), KAPPA,
                                            check_extent=False)
            st, q, _, _, l = O.propagate(p, None, L, BZ, KAPPA, check_extent=False,
                                         field=FieldMap(b0=BZ, h_max=0.01))
            assert st0 == O.OK and st == O.OK and l > 60.0, (st0, st, l)
            assert np.abs(q[:3] - q0[:3]).max() < 1e-8 and abs(l - l0) < 1e-8
            st1, q1, _, _, l1 = O.propagate(p, None, L, BZ, KAPPA, check_extent=False,
                                            field=replace(f, h_max=0.01))
            st2, q2, _, _, l2 = O.propagate(p, None, L, BZ, KAPPA, check_extent=False,
                                            field=replace(f, h_max=0.25))
            assert st1 == O.OK and st2 == O.OK
            assert np.abs(q1[:3] - q2[:3]).max() < 1e-8 and abs(l1 - l2) < 1e-8
            n += 1
    assert n == 12
