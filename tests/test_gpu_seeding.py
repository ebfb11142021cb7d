"""GPU parity of the combinatorial triplet seeding (mkf_make_seeds) against
the oracle's brute force over every hit triplet, and the seeds it makes used
for a find.  Needs an MI355X."""
import time

import numpy as np
import pytest

from oracle import oracle as O
from synth import SeedingConfig, barrel_endcap, generate, generate_event, make_batch, small_barrel

pytestmark = pytest.mark.gpu

WORKERS = 8  # event generation processes (sized for a 16-CPU host)

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


def make_ctx(M, w, b, flags=0):
    ctx = M.Context(w.find, flags=flags)
    ctx.load_geometry(w.layers)
    ctx.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v),
                  dev(b.layer))
    return ctx


def gpu_triplets(M, ctx, sc, cap):
    ev = torch.zeros(cap, dtype=torch.int32, device="cuda")
    hits = torch.zeros((cap, 3), dtype=torch.int32, device="cuda")
    t0 = time.time()
    n = ctx.make_seeds(sc, cap, ev, hits)
    return n, ev[:n].cpu().numpy(), hits[:n].cpu().numpy(), time.time() - t0


def check_event(w, sc, ev, g_hits, a_only=-1):
    """GPU triplets of one event (array [n][3]) against the oracle's brute
    force; differences only where the oracle puts a cut variable within
    1e-9 of its cut."""
    o, frag, n_near = O.triplet_seeds(w.find, sc, ev, a_only=a_only)
    gs = {tuple(t) for t in g_hits}
    os_ = {tuple(t) for t in o}
    assert len(gs) == len(g_hits), "duplicate triplets on the GPU"
    fr = {tuple(t) for t, f in zip(o, frag) if f}
    missing = os_ - gs - fr
    extra = gs - os_
    for t in extra:  # only near misses of the oracle may appear
        ok, margin, _ = O.triplet_params(w.find, sc, *[[ev.x[i], ev.y[i], ev.z[i]] for i in t])
        assert margin > -1e-9, (t, margin)
    assert not missing, sorted(missing)[:5]
    return len(os_), len(fr), len(extra)


def test_triplets_small_barrel_match_brute_force(mkf):
    w = small_barrel()
    b = generate(w)
    sc = SeedingConfig()
    ctx = make_ctx(mkf, w, b)
    n, ev, hits, _ = gpu_triplets(mkf, ctx, sc, 1 << 16)
    ctx.close()
    assert np.all(ev == 0)
    n_o, n_f, n_x = check_event(w, sc, b.events[0], hits)
    say("small barrel triplets", n, "oracle", n_o, "fragile", n_f, "extra", n_x)
    assert n >= 200


def test_triplets_realistic_events_match_brute_force(mkf):
    """Three events of 300 tracks with scattering, inefficiency and 30%
    noise, in one batch: every event's set equals the brute force."""
    w = barrel_endcap()
    evs = [generate_event(w, e, n_tracks=300) for e in range(3)]
    b = make_batch(evs)
    sc = SeedingConfig()
    ctx = make_ctx(mkf, w, b)
    n, ev, hits, _ = gpu_triplets(mkf, ctx, sc, 1 << 18)
    ctx.close()
    for e in range(3):
        n_o, n_f, n_x = check_event(w, sc, evs[e], hits[ev == e])
        say("event", e, "gpu", int((ev == e).sum()), "oracle", n_o, "fragile", n_f, "extra", n_x)


def test_triplets_capacity_error_reports_the_count(mkf):
    w = small_barrel()
    b = generate(w)
    ctx = make_ctx(mkf, w, b)
    n, _, _, _ = gpu_triplets(mkf, ctx, SeedingConfig(), 1 << 16)
    with pytest.raises(mkf.MkfError) as ei:
        gpu_triplets(mkf, ctx, SeedingConfig(), n - 1)
    assert ei.value.status == mkf.MKF_E_CAPACITY and str(n) in str(ei.value)
    with pytest.raises(mkf.MkfError) as ei:
        gpu_triplets(mkf, ctx, SeedingConfig(layers=(0, 1, 10)), 16)  # 10: not a barrel layer
    assert ei.value.status == mkf.MKF_E_ARG
    ctx.close()


def test_triplet_seeds_full_workload_and_find(mkf):
    """The benchmark's workload (100 events x 5,000 tracks): seeds from all
    triplets, 6 sampled first hits of 3 events checked against the brute
    force, and a batched find from those seeds finds the true track of
    nearly every particle that left a hit on each seeding layer."""
    w = barrel_endcap()
    b = generate(w, workers=WORKERS)
    sc = SeedingConfig()
    ctx = make_ctx(mkf, w, b, flags=mkf.F_BATCHED)
    cap = 4 << 20
    n, ev, hits, wall = gpu_triplets(mkf, ctx, sc, cap)
    say("triplets", n, "for", b.seed_hits.shape[0], "particles; wall", round(wall, 3), "s")
    rng = np.random.default_rng(44)
    for e in (0, 37, 99):  # the oracle takes ~3 s per first hit at this size
        E = b.events[e]
        cand = np.nonzero(E.layer == sc.layers[0])[0]
        g = hits[ev == e]
        for a in rng.choice(cand, 2, replace=False):
            check_event(w, sc, E, g[g[:, 0] == a], a_only=int(a))
    ctx.seed(dev(ev), dev(hits))
    ctx.find()
    tr = ctx.get_tracks(n)
    ctx.close()
    # efficiency: a particle with hits on the three seeding layers is found
    # if some track holds its first three hits and most of the rest
    eff_n = eff_d = 0
    for e in (0, 50):
        E = b.events[e]
        sel = np.nonzero(ev == e)[0]
        by_first = {}
        for s in sel:
            by_first.setdefault(tuple(hits[s]), []).append(s)
        for t, th in enumerate(E.track_hits):
            if len(th) < 6 or list(E.layer[th[:3]]) != list(sc.layers):
                continue
            if 1 / abs(E.truth_state[th[0]][3]) < 0.5:
                continue
            eff_d += 1
            for s in by_first.get(tuple(th[:3]), []):
                got = set(x for x in tr[s]["hit"] if x >= 0)
                if len(got & set(th[3:])) >= 0.7 * (len(th) - 3):
                    eff_n += 1
                    break
    say("efficiency for pT > 0.5 GeV/c:", eff_n, "/", eff_d)
    assert eff_n >= 0.97 * eff_d
