"""Pins of the oracle's region steering (Section 2.1: each tracking region
has a list of the layers the find traverses; five eta regions suffice for
CMS): the region a seed falls in and the plan it gets, the flag at a region
bound, and on simulated events that the five-region lists hold each seed's
own crossings in their order and find as many hits.  CPU only."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import Region, barrel_endcap, cms_like, five_regions, generate_event


def seed_inputs(ev, s):
    h = np.array([[ev.x[i], ev.y[i], ev.z[i]] for i in s], float).ravel()
    hv = np.array([[ev.var_u[i], ev.var_v[i]] for i in s], float).ravel()
    return h, hv, [int(ev.layer[i]) for i in s]


def eta_of(theta):
    return -np.log(np.tan(0.5 * theta))


@pytest.fixture(scope="module")
def case():
    w = barrel_endcap()
    ev = generate_event(w, 4, n_tracks=60)
    return w, ev


def test_plan_is_the_region_list_less_the_seed_layers(case):
    w, ev = case
    big = 1e30
    n = 0
    for s in ev.seeds[:40]:
        h, hv, hl = seed_inputs(ev, s)
        free = O.seed(w.find, w.layers, h, hv, hl)
        if not free["ok"]:
            continue
        eta = eta_of(free["par"][5])
        a = (27, 3, 9, 0, 14)          # any order, seed layers included
        b = (hl[2], 5, hl[0], 20)
        for st, want in (([Region(-big, eta - 0.05, a), Region(eta - 0.05, big, b)], (5, 20)),
                         ([Region(-big, eta + 0.05, a), Region(eta + 0.05, big, b)],
                          tuple(L for L in a if L not in hl)),
                         ([Region(eta + 0.05, big, b)], ())):
            r = O.seed(w.find, w.layers, h, hv, hl, steering=st)
            assert r["ok"] and not r["plan_fragile"]
            assert tuple(r["plan"]) == want
            # the seed state does not depend on the steering
            assert np.array_equal(r["par"], free["par"]) and np.array_equal(r["cov"], free["cov"])
        # a bound at the seed's eta (as FP32) is a fragile decision
        r = O.seed(w.find, w.layers, h, hv, hl,
                   steering=[Region(-big, float(np.float32(eta)), a)])
        assert r["plan_fragile"]
        n += 1
    assert n >= 30


def test_first_matching_region_wins(case):
    w, ev = case
    h, hv, hl = seed_inputs(ev, ev.seeds[0])
    st = [Region(-1e30, 1e30, (3, 4)), Region(-1e30, 1e30, (5, 6))]
    assert tuple(O.seed(w.find, w.layers, h, hv, hl, steering=st)["plan"]) == (3, 4)


def test_empty_plan_keeps_the_seed(case):
    """A seed in no region is found as its own seed state: its three hits
    and nothing more."""
    w, ev = case
    seeds = ev.seeds[:10]
    res = O.find_event(w.find, w.layers, ev, seeds=seeds, steering=[Region(50.0, 60.0, (3,))])
    for s, r in zip(seeds, res):
        h, hv, hl = seed_inputs(ev, s)
        sd = O.seed(w.find, w.layers, h, hv, hl)
        assert r["seed_ok"] == sd["ok"]
        if sd["ok"]:
            assert len(r["plan"]) == 0 and r["n_hits"] == 3 and r["n_miss"] == 0
            assert np.allclose(r["par"], sd["par"])


@pytest.mark.parametrize("make", [barrel_endcap, cms_like])
def test_five_regions_follow_the_crossings(make):
    """On a simulated event: each seed's helix plan (its crossings by path
    length) lies in its region's list in the same order for nearly every
    seed; the exceptions are barrel-region tracks that leave the barrel's
    end and meet a disk, which the barrel list does not hold.  The steered
    find takes as many hits as the find on the helix plans."""
    w = make()
    ev = generate_event(w, 1, n_tracks=300)
    st = five_regions()
    n = bad = 0
    for s in ev.seeds:
        h, hv, hl = seed_inputs(ev, s)
        a = O.seed(w.find, w.layers, h, hv, hl)
        b = O.seed(w.find, w.layers, h, hv, hl, steering=st)
        assert a["ok"] == b["ok"]
        if not a["ok"]:
            continue
        n += 1
        it = iter(list(b["plan"]))
        if not all(L in it for L in a["plan"]):
            bad += 1
            assert abs(eta_of(a["par"][5])) < 0.9          # the barrel region
            assert all(w.layers[L].kind == 1 for L in a["plan"] if L not in b["plan"])
    assert n > 250 and bad <= 0.05 * n
    free = O.find_event(w.find, w.layers, ev)
    steer = O.find_event(w.find, w.layers, ev, steering=st)
    same = sum(1 for x, y in zip(free, steer)
               if [k for k in x["hit"] if k >= 0] == [k for k in y["hit"] if k >= 0])
    hits_free = sum(x["n_hits"] for x in free)
    hits_steer = sum(x["n_hits"] for x in steer)
    assert same >= 0.95 * len(free)
    assert hits_steer >= 0.99 * hits_free
