"""GPU parity of the seed cleaning (mkf_clean_seeds) on dense jet-like
events seeded from every triplet: against the oracle's cleaning of its own
triplet seeds and seed fits, per triplet; and at the benchmark's size, the
find from the kept seeds.  Needs an MI355X."""
import time

import numpy as np
import pytest

from oracle import oracle as O
from synth import (CleaningConfig, SeedingConfig, barrel_endcap, generate, generate_event,
                   make_batch)

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


def seeded_ctx(M, w, b, cap, flags=0):
    ctx = M.Context(w.find, flags=flags)
    ctx.load_geometry(w.layers)
    ctx.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v),
                  dev(b.layer))
    ev = torch.zeros(cap, dtype=torch.int32, device="cuda")
    hits = torch.zeros((cap, 3), dtype=torch.int32, device="cuda")
    n = ctx.make_seeds(SeedingConfig(), cap, ev, hits)
    ev, hits = ev[:n].contiguous(), hits[:n].contiguous()
    ctx.seed(ev, hits)
    return ctx, ev, hits, n


def test_cleaning_dense_events_match_oracle(mkf):
    """Three jet-like events (300 tracks within 0.15 rad each)."""
    w = barrel_endcap()
    evs = [generate_event(w, e, n_tracks=300, phi_range=(0.0, 0.15)) for e in range(3)]
    b = make_batch(evs)
    cc = CleaningConfig()
    ctx, ev, hits, n = seeded_ctx(mkf, w, b, 1 << 18)
    keep = torch.full((n,), 7, dtype=torch.int32, device="cuda")
    nk = ctx.clean_seeds(cc, keep)
    keep = keep.cpu().numpy()
    g_ok = ctx.get_seed_states(n)[2]
    ctx.close()
    ev, hits = ev.cpu().numpy(), hits.cpu().numpy()
    assert nk == int(keep.sum()) and set(np.unique(keep)) <= {0, 1}
    assert np.all(keep[g_ok == 0] == 0)
    for e in range(3):
        E = evs[e]
        trip, _, _ = O.triplet_seeds(w.find, SeedingConfig(), E)
        fits = [O.seed(w.find, w.layers, np.array([[E.x[i], E.y[i], E.z[i]] for i in t]).ravel(),
                       np.array([[E.var_u[i], E.var_v[i]] for i in t]).ravel(),
                       [int(E.layer[i]) for i in t]) for t in trip]
        o_keep, o_frag = O.clean_seeds(trip, [f["ok"] for f in fits], [f["par"] for f in fits],
                                       [f["chi2"] for f in fits], cc.tol_ipt, cc.tol_eta,
                                       cc.tol_phi)
        sel = np.nonzero(ev == e)[0]
        g_idx = {tuple(hits[i]): i for i in sel}
        assert len(g_idx) == len(trip)
        fail = [(k, tuple(t)) for k, t in enumerate(trip)
                if not o_frag[k] and bool(keep[g_idx[tuple(t)]]) != bool(o_keep[k])]
        say("event", e, "seeds", len(trip), "kept", int(o_keep.sum()), "fragile",
            int(o_frag.sum()), "differ", len(fail))
        assert not fail, fail[:5]
        assert o_keep.sum() < 0.97 * len(trip)


def test_cleaned_seeds_full_workload(mkf):
    """The benchmark's workload seeded from every triplet: cleaning, then
    the batched find from the kept seeds only, against the find from all."""
    w = barrel_endcap()
    b = generate(w, workers=WORKERS)
    cc = CleaningConfig()
    ctx, ev, hits, n = seeded_ctx(mkf, w, b, 4 << 20, mkf.F_BATCHED)
    keep = torch.zeros(n, dtype=torch.int32, device="cuda")
    t0 = time.time()
    nk = ctx.clean_seeds(cc, keep)
    t_clean = time.time() - t0
    ctx.find()
    all_ms = ctx.stats()["find_ms"]
    sel = keep.bool()
    ctx.seed(ev[sel].contiguous(), hits[sel].contiguous())
    ctx.find()
    kept_ms = ctx.stats()["find_ms"]
    ctx.close()
    say("seeds", n, "kept", nk, "cleaning wall", round(t_clean, 3), "s; find ms all", all_ms,
        "kept", kept_ms)
    assert 0.5 * n < nk < n
