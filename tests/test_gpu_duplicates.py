"""GPU parity of duplicate-track removal (mkf_find_duplicates) after a find
seeded from every triplet: against the oracle's pipeline (its own triplet
seeds, find and removal), compared per seed triplet where both sides found
the same hits; and at the benchmark's size the rule checked on the GPU's
own tracks.  Needs an MI355X."""
import time

import numpy as np
import pytest

from oracle import oracle as O
from synth import SeedingConfig, barrel_endcap, generate, generate_event, make_batch, small_barrel

pytestmark = pytest.mark.gpu

WORKERS = 8  # event generation processes (sized for a 16-CPU host)
FRAC = 0.5

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def mkf():
    from paper_1811_04141_amd import mkf as M
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return M


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_pipeline(M, w, b, cap, flags=0):
    ctx = M.Context(w.find, flags=flags)
    ctx.load_geometry(w.layers)
    ctx.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v),
                  dev(b.layer))
    ev = torch.zeros(cap, dtype=torch.int32, device="cuda")
    hits = torch.zeros((cap, 3), dtype=torch.int32, device="cuda")
    n = ctx.make_seeds(SeedingConfig(), cap, ev, hits)
    ev, hits = ev[:n].contiguous(), hits[:n].contiguous()
    ctx.seed(ev, hits)
    ctx.find()
    tr = ctx.get_tracks(n)
    dup = torch.full((n,), 7, dtype=torch.int32, device="cuda")
    t0 = time.time()
    nd = ctx.find_duplicates(FRAC, dup)
    wall = time.time() - t0
    ctx.close()
    return ev.cpu().numpy(), hits.cpu().numpy(), tr, dup.cpu().numpy(), nd, wall


def gpu_sets(tr, hits):
    return [list(h) + [int(x) for x in t["hit"][:t["plan_len"]] if x >= 0] if t["status"] == 1
            else [] for t, h in zip(tr, hits)]


def compare_event(w, E, g_hits, g_tr, g_dup):
    trip, _, _ = O.triplet_seeds(w.find, SeedingConfig(), E)
    res = O.find_event(w.find, w.layers, E, seeds=trip)
    o_sets = O.track_hit_sets(res, trip)
    o_dup, o_frag = O.duplicates(o_sets, [r["chi2"] for r in res], trip, frac=FRAC)
    g_sets = gpu_sets(g_tr, g_hits)
    g_idx = {tuple(h): i for i, h in enumerate(g_hits)}
    assert len(g_idx) == len(trip) and all(tuple(t) in g_idx for t in trip)
    # seeds whose hit sets differ, and every track sharing a hit with one
    differ = {k for k, t in enumerate(trip) if sorted(o_sets[k]) != sorted(g_sets[g_idx[tuple(t)]])}
    by_hit = {}
    for k, s in enumerate(o_sets):
        for h in s:
            by_hit.setdefault(h, []).append(k)
    touched = set(differ)
    for k in differ:
        for h in o_sets[k]:
            touched.update(by_hit[h])
    out = {"n": len(trip), "dup": int(o_dup.sum()), "compared": 0, "differ": len(differ),
           "touched": len(touched), "fragile": int(o_frag.sum()), "fail": []}
    for k, t in enumerate(trip):
        if k in touched or o_frag[k]:
            continue
        out["compared"] += 1
        if bool(g_dup[g_idx[tuple(t)]]) != bool(o_dup[k]):
            out["fail"].append((k, tuple(t), bool(o_dup[k])))
    say({k: (v if k != "fail" else len(v)) for k, v in out.items()})
    assert not out["fail"], out["fail"][:5]
    return out


def test_duplicates_small_barrel_match_oracle(mkf):
    w = small_barrel()
    b = generate(w)
    ev, hits, tr, dup, nd, _ = gpu_pipeline(mkf, w, b, 1 << 16)
    assert nd == int(dup.sum()) and set(np.unique(dup)) <= {0, 1}
    out = compare_event(w, b.events[0], hits, tr, dup)
    assert out["compared"] >= 0.95 * out["n"] and out["dup"] > 0


def test_duplicates_realistic_events_match_oracle(mkf):
    """Three events of 300 tracks (scattering, inefficiency, 30% noise) in
    one batch, seeded from every triplet, both find forms."""
    w = barrel_endcap()
    evs = [generate_event(w, e, n_tracks=300) for e in range(3)]
    b = make_batch(evs)
    for flags in (0, mkf.F_BATCHED):
        ev, hits, tr, dup, nd, _ = gpu_pipeline(mkf, w, b, 1 << 18, flags)
        for e in range(3):
            sel = ev == e
            out = compare_event(w, evs[e], hits[sel], tr[sel], dup[sel])
            assert out["compared"] >= 0.9 * out["n"]


def test_duplicates_full_workload_follow_the_rule(mkf):
    """The benchmark's workload seeded from every triplet (~2.8 M seeds):
    in two events every kept track shares less than half of the shorter's
    hits with every other kept track, and every duplicate has a track
    ranking before it that shares at least that many."""
    w = barrel_endcap()
    b = generate(w, workers=WORKERS)
    ev, hits, tr, dup, nd, wall = gpu_pipeline(mkf, w, b, 4 << 20, mkf.F_BATCHED)
    say("tracks", len(tr), "duplicates", nd, "wall", round(wall, 3), "s")
    sets = gpu_sets(tr, hits)
    for e in (3, 71):
        idx = np.nonzero(ev == e)[0]
        by_hit = {}
        for i in idx:
            for h in sets[i]:
                by_hit.setdefault(h, []).append(i)

        def rank(i):
            return (-len(sets[i]), float(tr[i]["chi2"]), tuple(hits[i]))

        for i in idx:
            if not sets[i]:
                assert dup[i] == 0
                continue
            si = set(sets[i])
            partners = {u for h in sets[i] for u in by_hit[h] if u != i}
            conflicts = [u for u in partners
                         if len(si & set(sets[u])) >= FRAC * min(len(si), len(sets[u]))]
            better = [u for u in conflicts if rank(u) < rank(i)]
            assert bool(dup[i]) == bool(better), (i, sets[i])
