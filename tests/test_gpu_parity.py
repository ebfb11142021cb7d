"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.  Needs an MI355X."""
import os
import sys
import time

import numpy as np
import pytest

from oracle import oracle as O
from synth import (BARREL, FindConfig, Layer, barrel_endcap, generate, generate_event,
                   make_batch, small_barrel)
import parity as PT

pytestmark = pytest.mark.gpu

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


def run_find(M, w, batch, flags=0, fc=None):
    ctx = M.Context(fc or w.find, flags=flags)
    ctx.load_geometry(w.layers)
    ctx.load_hits(batch.ev_off, dev(batch.x), dev(batch.y), dev(batch.z), dev(batch.var_u),
                  dev(batch.var_v), dev(batch.layer))
    ctx.seed(dev(batch.seed_event), dev(batch.seed_hits))
    ctx.find()
    n = batch.seed_hits.shape[0]
    tr = ctx.get_tracks(n)
    seeds = ctx.get_seed_states(n)
    st = ctx.stats()
    ctx.close()
    return tr, seeds, st


def check(out, max_div_frac=0.05):
    say({k: (v if k != "fail" else len(v)) for k, v in out.items()})
    assert not out["fail"], out["fail"][:5]
    assert out["tie_diverged"] + out["plan_diverged"] <= max_div_frac * out["n"] + 1


# ----------------------------------------------------------- propagation

def test_propagate_matches_oracle(mkf):
    w = barrel_endcap()
    rng = np.random.default_rng(21)
    n = 4096
    ev = generate_event(w, 0, n_tracks=2000)
    # start from true states at recorded hits, go to a random other layer
    idx = rng.choice(np.nonzero(ev.track >= 0)[0], n)
    par = ev.truth_state[idx].astype(np.float32)
    A = rng.normal(size=(n, 6, 6)) * np.array([1e-2, 1e-2, 1e-2, 1e-3, 1e-3, 1e-3])
    full = np.einsum("nij,nkj->nik", A, A) + np.diag([1e-4, 1e-4, 1e-4, 1e-6, 1e-6, 1e-6])
    cov = mkf.pack_cov(full).astype(np.float32)
    layer = rng.integers(0, len(w.layers), n).astype(np.int32)
    ctx = mkf.Context(w.find)
    ctx.load_geometry(w.layers)
    o_par = torch.zeros((n, 6), device="cuda")
    o_cov = torch.zeros((n, 21), device="cuda")
    o_l = torch.zeros(n, device="cuda")
    o_st = torch.zeros(n, dtype=torch.int32, device="cuda")
    ctx.propagate(dev(par), dev(cov), dev(layer), o_par, o_cov, o_l, o_st)
    torch.cuda.synchronize()
    g_par, g_cov, g_l, g_st = (t.cpu().numpy() for t in (o_par, o_cov, o_l, o_st))
    ctx.close()
    n_ok = n_edge = 0
    fc = w.find
    for i in range(n):
        L = w.layers[layer[i]]
        st, pp, Cp, _, l = O.propagate(par[i].astype(float), mkf.unpack_cov(cov[i]).astype(float),
                                       L, fc.bz, fc.kappa, fc.l_min, fc.edge_margin, True)
        if st != g_st[i]:
            # only allowed where the crossing sits on a widened edge
            st2, pp2, _, _, _ = O.propagate(par[i].astype(float), None, L, fc.bz, fc.kappa,
                                            fc.l_min, 0.0, False)
            q = pp2[2] if L.kind == BARREL else np.hypot(pp2[0], pp2[1])
            edge = min(abs(q - (L.ext_lo - fc.edge_margin)), abs(q - (L.ext_hi + fc.edge_margin)))
            assert st2 == O.OK and edge < 1e-3, (i, st, g_st[i])
            n_edge += 1
            continue
        if st != O.OK:
            continue
        n_ok += 1
        ok, rel = PT.par_ok(g_par[i], pp)
        assert ok, (i, rel)
        assert abs(g_l[i] - l) <= 1e-5 * max(l, 1.0), (g_l[i], l)
        assert PT.cov_ok(mkf.unpack_cov(g_cov[i]), Cp), i
    say("propagated", n_ok, "edge flips", n_edge)
    assert n_ok > n // 8


# --------------------------------------------------------------- seeding

@pytest.mark.parametrize("wname", ["small", "realistic"])
def test_seed_states_match_oracle(mkf, wname):
    w = small_barrel() if wname == "small" else barrel_endcap()
    ev = generate_event(w, 0, n_tracks=None if wname == "small" else 1000)
    b = make_batch([ev])
    ctx = mkf.Context(w.find)
    ctx.load_geometry(w.layers)
    ctx.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v), dev(b.layer))
    ctx.seed(dev(b.seed_event), dev(b.seed_hits))
    par, cov, ok, plen, plan, chi2 = ctx.get_seed_states(b.seed_hits.shape[0])
    ctx.close()
    bad = 0
    for s in range(b.seed_hits.shape[0]):
        sh = b.seed_hits[s]
        h = np.array([[ev.x[i], ev.y[i], ev.z[i]] for i in sh], float).ravel()
        hv = np.array([[ev.var_u[i], ev.var_v[i]] for i in sh], float).ravel()
        r = O.seed(w.find, w.layers, h, hv, [int(ev.layer[i]) for i in sh], pos_tol=1e-3)
        assert bool(ok[s]) == r["ok"]
        if not r["ok"]:
            continue
        good, rel = PT.par_ok(par[s], r["par"])
        assert good, (s, rel)
        assert PT.cov_ok(mkf.unpack_cov(cov[s]), r["cov"]), s
        assert PT.chi2_ok(chi2[s], r["chi2"]), (s, chi2[s], r["chi2"])
        if list(plan[s, :plen[s]]) != list(r["plan"]):
            assert r["plan_fragile"], (s, plan[s, :plen[s]], r["plan"])
            bad += 1
    assert bad <= 0.01 * b.seed_hits.shape[0] + 1


# --------------------------------------------------------------- finding

def test_find_small_barrel_matches_oracle_exactly(mkf):
    w = small_barrel()
    b = generate(w)
    tr, _, st = run_find(mkf, w, b)
    ref = O.find_event(w.find, w.layers, b.events[0])
    out = PT.compare_tracks(tr, ref, mkf.unpack_cov)
    check(out, max_div_frac=0.0)
    assert out["equal"] == len(ref)
    assert st["n_steps"] == sum(r["n_steps"] for r in ref)


@pytest.mark.parametrize("flags", [0, 1])
def test_find_realistic_events_match_oracle(mkf, flags):
    """Two realistic events of 5,000 tracks (scattering, inefficiency, 30%
    noise) found on the GPU in full; the oracle recomputes a sample of
    seeds one by one."""
    w = barrel_endcap()
    b = generate(w, events=[0, 1])
    t0 = time.time()
    tr, _, st = run_find(mkf, w, b, flags=flags)
    say("gpu find ms", st["find_ms"], "steps", st["n_steps"], "wall", time.time() - t0)
    rng = np.random.default_rng(5)
    for e in range(2):
        sel = np.nonzero(b.seed_event == e)[0]
        pick = np.sort(rng.choice(sel, 120, replace=False))
        local = pick - sel[0]
        ref = O.find_event(w.find, w.layers, b.events[e], seeds=b.events[e].seeds[local])
        check(PT.compare_tracks(tr[pick], ref, mkf.unpack_cov))


@pytest.mark.parametrize("n_cand", [6, 8, 3])
def test_batched_equals_layer_synchronous_bitwise(mkf, n_cand):
    """The persistent form (6-lane seed groups for budgets up to 6, else 8)
    and the layer-synchronous form (the same lane groups) give the same bytes."""
    import dataclasses
    w = barrel_endcap()
    fc = dataclasses.replace(w.find, n_cand=n_cand)
    b = generate(w, events=[2, 3, 4])
    a, _, sa = run_find(mkf, w, b, flags=0, fc=fc)
    c, _, sc = run_find(mkf, w, b, flags=1, fc=fc)
    assert sa["n_steps"] == sc["n_steps"]
    assert a.tobytes() == c.tobytes()


def test_launch_shapes_do_not_change_results(mkf, tmp_path):
    """Every persistent-kernel launch shape and hit-index binning the
    autotuner may pick (waves per SIMD, blocks per CU, 6- or 8-lane seed
    groups, bin counts halved to quadrupled) gives bitwise the same tracks,
    in both find forms; the autotuner's cache round-trips."""
    w = barrel_endcap()
    b = generate(w, events=[5, 6])
    ctx = mkf.Context(w.find, flags=mkf.F_BATCHED)
    ctx.load_geometry(w.layers)
    ctx.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v),
                  dev(b.layer))
    ctx.seed(dev(b.seed_event), dev(b.seed_hits))
    n = b.seed_hits.shape[0]
    ref = None
    shapes = [(2, 8, 0, 0, 0), (1, 1, 6, 0, 0), (3, 3, 6, 0, 0), (4, 8, 6, 0, 0),
              (1, 2, 8, 0, 0), (2, 4, 8, 0, 0), (3, 6, 8, 0, 0), (4, 4, 8, 0, 0),
              (3, 3, 6, -1, 1), (3, 3, 6, 1, -1), (2, 2, 8, 2, 2), (3, 3, 6, -2, -2)]
    for shape in shapes:
        print("shape", shape, flush=True)
        ctx.set_tuning(*shape)
        assert ctx.get_tuning() == dict(zip(("waves_per_simd", "blocks_per_cu", "lane_group",
                                             "phi_bin_shift", "q_bin_shift"), shape))
        ctx.find()
        tr = ctx.get_tracks(n)
        ref = tr if ref is None else ref
        assert tr.tobytes() == ref.tobytes(), shape
    # the layer-synchronous form on a rebinned index
    c2 = mkf.Context(w.find)
    c2.load_geometry(w.layers)
    c2.set_tuning(2, 8, 0, 1, -1)
    c2.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v),
                 dev(b.layer))
    c2.seed(dev(b.seed_event), dev(b.seed_hits))
    c2.find()
    assert c2.get_tracks(n).tobytes() == ref.tobytes()
    c2.set_tuning(2, 8, 0, -1, 2)  # rebuilt with the hits loaded
    c2.find()
    assert c2.get_tracks(n).tobytes() == ref.tobytes()
    c2.close()
    cache = str(tmp_path / "tune.txt")
    t1 = ctx.autotune(repeats=1, cache_path=cache)
    print("autotuned", t1, flush=True)
    t2 = ctx.autotune(repeats=1, cache_path=cache)
    assert t1 == t2 and open(cache).read().count("\n") == 1
    assert ctx.get_tuning() == t1
    ctx.find()
    assert ctx.get_tracks(n).tobytes() == ref.tobytes()
    with pytest.raises(mkf.MkfError):
        ctx.set_tuning(2, 8, 7, 0, 0)
    with pytest.raises(mkf.MkfError):
        ctx.set_tuning(2, 8, 0, 3, 0)
    ctx.close()


def test_find_edge_cases(mkf):
    """An event without hits, an event whose seeds have empty plans, seeds
    with a candidate budget of one, and no seeds at all."""
    w = small_barrel()
    ev = generate_event(w, 0)
    # seeds on the three outermost layers: nothing left to cross
    outer = np.array([h[-3:] for h in ev.track_hits[:20]], np.int32)
    from synth.events import Event
    ev2 = Event(ev.x, ev.y, ev.z, ev.var_u, ev.var_v, ev.layer, ev.track, outer,
                ev.seed_track[:20], ev.truth_state, ev.track_hits)
    empty = Event(*(a[:0] for a in (ev.x, ev.y, ev.z, ev.var_u, ev.var_v, ev.layer, ev.track)),
                  np.zeros((0, 3), np.int32), np.zeros(0, np.int32), ev.truth_state[:0], [])
    b = make_batch([ev2, empty])
    tr, _, st = run_find(mkf, w, b)
    ref = O.find_event(w.find, w.layers, ev2)
    check(PT.compare_tracks(tr, ref, mkf.unpack_cov), max_div_frac=0.0)
    assert tr.shape[0] == 20
    fc1 = FindConfig(ms_sigma=0.0, n_cand=1)
    b1 = make_batch([ev])
    tr1, _, _ = run_find(mkf, w, b1, fc=fc1)
    ref1 = O.find_event(fc1, w.layers, ev)
    check(PT.compare_tracks(tr1, ref1, mkf.unpack_cov), max_div_frac=0.0)
    # no seeds
    b0 = make_batch([ev])
    b0.seed_event = b0.seed_event[:0]
    b0.seed_hits = b0.seed_hits[:0]
    tr0, _, st0 = run_find(mkf, w, b0)
    assert tr0.shape[0] == 0 and st0["n_steps"] == 0


def test_find_maximum_layers_and_plan(mkf):
    """The largest geometry the library takes (32 cylinders) with plans of
    29 layers: the oracle on every seed, and the two forms bitwise equal
    (the persistent form sizes its LDS records by the longest plan)."""
    from synth import EventRecipe, Workload
    from synth.workloads import SIGMA_RPHI, SIGMA_Z
    radii = np.linspace(3.0, 100.0, 32)
    layers = [Layer(BARREL, float(r), -200.0, 200.0, SIGMA_RPHI ** 2, SIGMA_Z ** 2) for r in radii]
    w = Workload(name="barrel32_1x400", layers=tuple(layers),
                 recipe=EventRecipe(pt_lo=1.0, pt_hi=10.0, eta_max=1.0, ms_sigma=0.001,
                                    hit_ineff=0.02, noise_frac=0.3),
                 find=FindConfig(), n_events=1, n_tracks=(400, 400), master_seed=0x5EED0007)
    b = generate(w)
    a, seeds, sa = run_find(mkf, w, b, flags=0)
    c, _, sc = run_find(mkf, w, b, flags=mkf.F_BATCHED)
    plen = seeds[3]
    say("plan lengths: max", plen.max(), "mean", plen.mean())
    assert plen.max() == 29
    assert sa["n_steps"] == sc["n_steps"] and a.tobytes() == c.tobytes()
    ref = O.find_event(w.find, w.layers, b.events[0])
    check(PT.compare_tracks(a, ref, mkf.unpack_cov))


# ------------------------------------------------------------------- fit

def test_fit_matches_oracle(mkf):
    w = barrel_endcap()
    fc = w.find
    ev = generate_event(w, 9, n_tracks=3000)
    tracks = [h for h in ev.track_hits if h.shape[0] >= 6]
    n = len(tracks)
    n_steps = max(h.shape[0] for h in tracks) - 3
    kind = np.zeros((n_steps, n), np.int8)
    pos = np.zeros((n_steps, n), np.float32)
    X = np.zeros((6, n_steps, n), np.float32)
    length = np.zeros(n, np.int32)
    init_par = np.zeros((n, 6), np.float32)
    init_cov = np.zeros((n, 21), np.float32)
    for t, h in enumerate(tracks):
        hh = np.array([[ev.x[i], ev.y[i], ev.z[i]] for i in h[:3]], float).ravel()
        hv = np.array([[ev.var_u[i], ev.var_v[i]] for i in h[:3]], float).ravel()
        sd = O.seed(fc, w.layers, hh, hv, [int(ev.layer[i]) for i in h[:3]])
        init_par[t] = sd["par"]
        from paper_1811_04141_amd.mkf import pack_cov
        init_cov[t] = pack_cov(sd["cov"])
        rest = h[3:]
        length[t] = rest.shape[0]
        for k, i in enumerate(rest):
            L = w.layers[ev.layer[i]]
            kind[k, t], pos[k, t] = L.kind, L.pos
            X[:, k, t] = [ev.x[i], ev.y[i], ev.z[i], ev.var_u[i], ev.var_v[i], 0]
    ctx = mkf.Context(fc)
    outs = [torch.zeros((n, 6), device="cuda"), torch.zeros((n, 21), device="cuda"),
            torch.zeros(n, device="cuda"), torch.zeros(n, dtype=torch.int32, device="cuda")]
    ctx.fit(dev(kind), dev(pos), dev(X[0]), dev(X[1]), dev(X[2]), dev(X[3]), dev(X[4]),
            dev(length), dev(init_par), dev(init_cov), *outs)
    torch.cuda.synchronize()
    g_par, g_cov, g_chi, g_st = (o.cpu().numpy() for o in outs)
    ctx.close()
    worst = worst_graze = 0.0
    n_graze = 0
    for t in range(n):
        rest = tracks[t][3:]
        rc, p, Cm, c2 = O.fit_track(fc, init_par[t].astype(float),
                                    mkf.unpack_cov(init_cov[t]).astype(float),
                                    kind[:length[t], t].astype(np.int32),
                                    pos[:length[t], t].astype(float),
                                    X[:3, :length[t], t].T.astype(float),
                                    X[3, :length[t], t].astype(float),
                                    X[4, :length[t], t].astype(float))
        assert (rc == 0) == (g_st[t] == 0)
        if rc:
            continue
        ok, rel = PT.par_ok(g_par[t], p)
        assert ok, (t, rel)
        assert PT.chi2_ok(g_chi[t], c2), (g_chi[t], c2)
        # conditioning: the smallest cosine between track and surface normal
        # over the crossings; the surface projection divides by it
        cmin = 1.0
        for i in rest:
            s = ev.truth_state[i]
            d = np.array([np.cos(s[4]), np.sin(s[4]), 1 / np.tan(s[5])])
            nrm = (np.array([s[0], s[1], 0.0]) if w.layers[ev.layer[i]].kind == BARREL
                   else np.array([0.0, 0.0, 1.0]))
            cmin = min(cmin, abs(d @ nrm) / np.linalg.norm(d) / np.linalg.norm(nrm))
        ce = PT.cov_err(mkf.unpack_cov(g_cov[t]), Cm)
        if cmin >= PT.GRAZING_COS:
            worst = max(worst, ce)
            assert ce <= PT.COV_REL_FOUND, (t, ce, cmin)
        else:
            n_graze += 1
            worst_graze = max(worst_graze, ce)
            assert ce <= PT.COV_REL_GRAZING, (t, ce, cmin)
    say("fit: worst covariance error (correlation units)", worst, "grazing tracks", n_graze,
        "worst there", worst_graze)


def test_repeated_finds_and_graph_replays_are_bitwise_identical(mkf):
    """Results never depend on which wave claims which tile: three finds of
    the persistent form and five replays of its captured graph, with other
    GPU work between the replays, give the same bytes and step counts."""
    w = barrel_endcap()
    b = generate(w, events=[7, 8])
    n = b.seed_hits.shape[0]
    ref = None
    for flags, times in ((mkf.F_BATCHED, 3), (mkf.F_BATCHED | mkf.F_GRAPH, 5)):
        stream = torch.cuda.Stream()
        ctx = mkf.Context(w.find, flags=flags, stream=stream.cuda_stream)
        try:
            ctx.load_geometry(w.layers)
            ctx.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v),
                          dev(b.layer))
            ctx.seed(dev(b.seed_event), dev(b.seed_hits))
            for i in range(times):
                ctx.find()
                tr, st = ctx.get_tracks(n), ctx.stats()
                if ref is None:
                    ref = (tr, st["n_steps"])
                assert tr.tobytes() == ref[0].tobytes(), (flags, i)
                assert st["n_steps"] == ref[1], (flags, i)
                x = torch.randn(1 << 20, device="cuda")  # other work between finds
                assert torch.isfinite((x * 2.0).sum()).item()
        finally:
            ctx.close()
