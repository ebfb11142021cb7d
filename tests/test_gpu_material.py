"""GPU parity with a material map (mkf_load_material): seed states, both
find forms, the backward fit and smoothing of the found tracks, and the
search-free fit, against the oracle with the same map; clearing the map
gives back the constant-angle results; host-side validation.  Needs an
MI355X."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import (BARREL, barrel_material, cms_like_material, generate, generate_event,
                   make_batch)
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


def context(M, w, b, flags=0, material=True):
    ctx = M.Context(w.find, flags=flags)
    ctx.load_geometry(w.layers)
    if material:
        ctx.load_material(w.material)
    ctx.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v),
                  dev(b.layer))
    ctx.seed(dev(b.seed_event), dev(b.seed_hits))
    return ctx


def seed_inputs(E, sh):
    h = np.array([[E.x[j], E.y[j], E.z[j]] for j in sh], float).ravel()
    hv = np.array([[E.var_u[j], E.var_v[j]] for j in sh], float).ravel()
    return h, hv, [int(E.layer[j]) for j in sh]


def test_seed_states_with_material_match_oracle(mkf):
    w = cms_like_material()
    ev = generate_event(w, 2, n_tracks=800)
    b = make_batch([ev])
    ctx = context(mkf, w, b)
    par, cov, ok, plen, plan, chi2 = ctx.get_seed_states(b.seed_hits.shape[0])
    ctx.close()
    worst = 0.0
    for s in range(b.seed_hits.shape[0]):
        h, hv, hl = seed_inputs(ev, b.seed_hits[s])
        r = O.seed(w.find, w.layers, h, hv, hl, pos_tol=1e-3, material=w.material)
        assert bool(ok[s]) == r["ok"]
        if not r["ok"]:
            continue
        assert PT.par_ok(par[s], r["par"])[0], s
        assert PT.chi2_ok(chi2[s], r["chi2"]), (chi2[s], r["chi2"])
        worst = max(worst, PT.cov_err(mkf.unpack_cov(cov[s]), r["cov"]))
    say("seeds", b.seed_hits.shape[0], "worst covariance", worst)
    assert worst < PT.COV_REL_GRAZING


@pytest.mark.parametrize("flags", [0, 1])
def test_find_with_material_matches_oracle(mkf, flags):
    w = cms_like_material()
    b = generate(w, events=[0, 1])
    ctx = context(mkf, w, b, flags)
    ctx.find()
    n = b.seed_hits.shape[0]
    tr = ctx.get_tracks(n)
    bf = [torch.zeros((n, 6), device="cuda"), torch.zeros((n, 21), device="cuda"),
          torch.zeros(n, device="cuda"), torch.zeros(n, dtype=torch.int32, device="cuda")]
    ctx.backward_fit(*bf)
    ns = O.MAX_PLAN + 1
    sm = [torch.zeros((n, ns, 6), device="cuda"), torch.zeros((n, ns, 21), device="cuda"),
          torch.zeros(n, dtype=torch.int32, device="cuda")]
    ctx.smooth(*sm)
    torch.cuda.synchronize()
    bf = [a.cpu().numpy() for a in bf]
    sm = [a.cpu().numpy() for a in sm]
    ctx.close()
    rng = np.random.default_rng(93)
    worst_bf = worst_sm = 0.0
    for e in range(2):
        E = b.events[e]
        sel = np.nonzero(b.seed_event == e)[0]
        pick = np.sort(rng.choice(sel, 120, replace=False))
        seeds = E.seeds[pick - sel[0]]
        ref = O.find_event(w.find, w.layers, E, seeds=seeds, material=w.material)
        out = PT.compare_tracks(tr[pick], ref, mkf.unpack_cov)
        say({k: (v if k != "fail" else len(v)) for k, v in out.items()})
        assert not out["fail"], out["fail"][:5]
        assert out["equal"] >= 0.9 * out["n"]
        for k, (i, r) in enumerate(zip(pick, ref)):
            if not r["seed_ok"] or list(tr[i]["hit"][:len(r["plan"])]) != list(r["hit"]):
                continue
            st, p, Cm, c2, _ = O.backward_fit(w.find, w.layers, E, seeds[k], r,
                                              material=w.material)
            assert bf[3][i] == st
            if st == 1:
                assert PT.par_ok(bf[0][i], p)[0] and PT.chi2_ok(bf[2][i], c2), (i, bf[0][i], p)
                worst_bf = max(worst_bf, PT.cov_err(mkf.unpack_cov(bf[1][i]), Cm))
            h, hv, hl = seed_inputs(E, seeds[k])
            sd = O.seed(w.find, w.layers, h, hv, hl, material=w.material)
            m, _, sp, sc = O.smooth_track(w.find, w.layers, E, hl[2], sd["par"], sd["cov"], r,
                                          material=w.material)
            assert sm[2][i] == m
            for q in range(max(m, 0)):
                assert PT.par_ok(sm[0][i, q], sp[q])[0], (i, q)
                worst_sm = max(worst_sm, PT.cov_err(mkf.unpack_cov(sm[1][i, q]), sc[q]))
    say("worst covariance: backward fit", worst_bf, "smoothing", worst_sm)
    assert worst_bf < PT.COV_REL_GRAZING and worst_sm < PT.COV_REL_GRAZING


def test_fit_with_material_matches_oracle(mkf):
    """Search-free fit of simulated tracks through heavy material."""
    w = barrel_material(n_tracks=600)
    fc = w.find
    ev = generate_event(w, 3)
    tracks = [h for h in ev.track_hits if h.shape[0] >= 6]
    n = len(tracks)
    n_steps = max(h.shape[0] for h in tracks) - 3
    kind = np.zeros((n_steps, n), np.int8)
    pos = np.zeros((n_steps, n), np.float32)
    X = np.zeros((5, n_steps, n), np.float32)
    length = np.zeros(n, np.int32)
    init_par = np.zeros((n, 6), np.float32)
    init_cov = np.zeros((n, 21), np.float32)
    for t, h in enumerate(tracks):
        hh, hv, hl = seed_inputs(ev, h[:3])
        sd = O.seed(fc, w.layers, hh, hv, hl, material=w.material)
        init_par[t] = sd["par"]
        init_cov[t] = mkf.pack_cov(sd["cov"])
        rest = h[3:]
        length[t] = rest.shape[0]
        for k, i in enumerate(rest):
            L = w.layers[ev.layer[i]]
            kind[k, t], pos[k, t] = L.kind, L.pos
            X[:, k, t] = [ev.x[i], ev.y[i], ev.z[i], ev.var_u[i], ev.var_v[i]]
    ctx = mkf.Context(fc)
    ctx.load_material(w.material)
    outs = [torch.zeros((n, 6), device="cuda"), torch.zeros((n, 21), device="cuda"),
            torch.zeros(n, device="cuda"), torch.zeros(n, dtype=torch.int32, device="cuda")]
    ctx.fit(dev(kind), dev(pos), dev(X[0]), dev(X[1]), dev(X[2]), dev(X[3]), dev(X[4]),
            dev(length), dev(init_par), dev(init_cov), *outs)
    torch.cuda.synchronize()
    g_par, g_cov, g_chi, g_st = (o.cpu().numpy() for o in outs)
    ctx.close()
    worst = 0.0
    for t in range(n):
        m = length[t]
        rc, p, Cm, c2 = O.fit_track(fc, init_par[t].astype(float),
                                    mkf.unpack_cov(init_cov[t]).astype(float),
                                    kind[:m, t].astype(np.int32), pos[:m, t].astype(float),
                                    X[:3, :m, t].T.astype(float), X[3, :m, t].astype(float),
                                    X[4, :m, t].astype(float), material=w.material)
        assert (rc == 0) == (g_st[t] == 0)
        if rc:
            continue
        ok, rel = PT.par_ok(g_par[t], p)
        assert ok, (t, rel)
        assert PT.chi2_ok(g_chi[t], c2), (g_chi[t], c2)
        worst = max(worst, PT.cov_err(mkf.unpack_cov(g_cov[t]), Cm))
    say("fit tracks", n, "worst covariance", worst)
    assert n > 400 and worst < PT.COV_REL_GRAZING


def test_cleared_map_gives_the_constant_angle_results(mkf):
    w = cms_like_material()
    b = generate(w, events=[0])
    ref = context(mkf, w, b, material=False)
    ref.find()
    n = b.seed_hits.shape[0]
    a = ref.get_tracks(n)
    ref.close()
    ctx = context(mkf, w, b)
    ctx.find()
    with_map = ctx.get_tracks(n)
    ctx.load_material(None)
    ctx.seed(dev(b.seed_event), dev(b.seed_hits))
    ctx.find()
    c = ctx.get_tracks(n)
    ctx.close()
    assert a.tobytes() == c.tobytes()
    assert a.tobytes() != with_map.tobytes()


def test_bad_material_is_an_argument_error(mkf):
    from dataclasses import replace
    w = cms_like_material()
    m = w.material
    ctx = mkf.Context(w.find)
    for bad in (replace(m, n_r=0), replace(m, r_max=-1.0), replace(m, mass=0.0),
                replace(m, k_max=0.5), replace(m, x_x0=m.x_x0 * np.float32(np.nan)),
                replace(m, xi=m.xi - np.float32(1.0))):
        with pytest.raises((mkf.MkfError, ValueError)) as ei:
            ctx.load_material(bad)
        if isinstance(ei.value, mkf.MkfError):
            assert ei.value.status == mkf.MKF_E_ARG
    ctx.close()


def test_surrogate_with_material_map_keeps_the_hit_lists(mkf):
    """The surrogate form with a material map: the network only starts the
    barrel crossings (one Newton step checks each hint), the material update
    follows as without it, so the hit lists are those of the form without
    the surrogate and most hints are kept."""
    w = cms_like_material()
    b = generate(w, events=[0, 1])
    n = b.seed_hits.shape[0]
    ref = context(mkf, w, b, flags=mkf.F_BATCHED)
    ref.find()
    tp = ref.get_tracks(n)
    ref.close()
    ctx = context(mkf, w, b, flags=mkf.F_BATCHED | mkf.F_SURROGATE)
    try:
        rep = ctx.surrogate_train(n_samples=1 << 20, epochs=4, batch=512, lr=3e-3, seed=23,
                                  loss_w=(1, .01, .01, .01, .01, .01, .01))
        say("training", rep)
        ctx.find()
        ts = ctx.get_tracks(n)
        st = ctx.stats()
    finally:
        ctx.close()
    kept, rej = st["sur_kept"], st["sur_rejected"]
    same = np.all(ts["hit"] == tp["hit"], axis=1).mean()
    say("kept", kept, "rejected", rej, "same hit lists", same)
    assert kept >= 0.5 * (kept + rej)
    assert same >= 0.995
