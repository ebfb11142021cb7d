"""GPU parity in a parameterised field (mkf_load_field): single
propagations, seed states, both find forms, the backward fit and smoothing
of the found tracks against the oracle in the same solenoid-like field;
clearing the field gives back the uniform-field results; host-side
validation.  Needs an MI355X."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import BARREL, barrel_endcap_field, generate, generate_event, make_batch
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


def context(M, w, b, flags=0, field=True):
    ctx = M.Context(w.find, flags=flags)
    ctx.load_geometry(w.layers)
    if field:
        ctx.load_field(w.field)
    ctx.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v),
                  dev(b.layer))
    ctx.seed(dev(b.seed_event), dev(b.seed_hits))
    return ctx


def seed_inputs(E, sh):
    h = np.array([[E.x[j], E.y[j], E.z[j]] for j in sh], float).ravel()
    hv = np.array([[E.var_u[j], E.var_v[j]] for j in sh], float).ravel()
    return h, hv, [int(E.layer[j]) for j in sh]


def test_propagate_in_the_field_matches_oracle(mkf):
    """True states at recorded hits, each carried to a random layer."""
    w = barrel_endcap_field()
    fc = w.find
    rng = np.random.default_rng(31)
    n = 2048
    ev = generate_event(w, 0, n_tracks=1000)
    idx = rng.choice(np.nonzero(ev.track >= 0)[0], n)
    par = ev.truth_state[idx].astype(np.float32)
    A = rng.normal(size=(n, 6, 6)) * np.array([1e-2, 1e-2, 1e-2, 1e-3, 1e-3, 1e-3])
    full = np.einsum("nij,nkj->nik", A, A) + np.diag([1e-4, 1e-4, 1e-4, 1e-6, 1e-6, 1e-6])
    cov = mkf.pack_cov(full).astype(np.float32)
    layer = rng.integers(0, len(w.layers), n).astype(np.int32)
    ctx = mkf.Context(fc)
    ctx.load_geometry(w.layers)
    ctx.load_field(w.field)
    o = [torch.zeros((n, 6), device="cuda"), torch.zeros((n, 21), device="cuda"),
         torch.zeros(n, device="cuda"), torch.zeros(n, dtype=torch.int32, device="cuda")]
    ctx.propagate(dev(par), dev(cov), dev(layer), *o)
    torch.cuda.synchronize()
    g_par, g_cov, g_l, g_st = (t.cpu().numpy() for t in o)
    ctx.close()
    n_ok = n_edge = 0
    for i in range(n):
        L = w.layers[layer[i]]
        st, pp, Cp, _, l = O.propagate(par[i].astype(float), mkf.unpack_cov(cov[i]).astype(float),
                                       L, fc.bz, fc.kappa, fc.l_min, fc.edge_margin, True,
                                       field=w.field)
        if st != g_st[i]:
            st2, pp2, _, _, _ = O.propagate(par[i].astype(float), None, L, fc.bz, fc.kappa,
                                            fc.l_min, 0.0, False, field=w.field)
            q = pp2[2] if L.kind == BARREL else np.hypot(pp2[0], pp2[1])
            edge = min(abs(q - (L.ext_lo - fc.edge_margin)), abs(q - (L.ext_hi + fc.edge_margin)))
            assert st2 == O.OK and edge < 1e-3, (i, st, g_st[i])
            n_edge += 1
            continue
        if st != O.OK:
            continue
        n_ok += 1
        ok, rel = PT.par_ok(g_par[i], pp)
        assert ok, (i, rel, g_par[i], pp)
        assert abs(g_l[i] - l) <= 1e-5 * max(l, 1.0), (g_l[i], l)
        assert PT.cov_ok(mkf.unpack_cov(g_cov[i]), Cp), i
    say("propagations", n, "equal", n_ok, "edge", n_edge)
    assert n_ok > 300 and n_edge <= 2


def test_seed_states_in_the_field_match_oracle(mkf):
    w = barrel_endcap_field()
    ev = generate_event(w, 2, n_tracks=800)
    b = make_batch([ev])
    ctx = context(mkf, w, b)
    par, cov, ok, plen, plan, chi2 = ctx.get_seed_states(b.seed_hits.shape[0])
    ctx.close()
    worst = 0.0
    for s in range(b.seed_hits.shape[0]):
        h, hv, hl = seed_inputs(ev, b.seed_hits[s])
        r = O.seed(w.find, w.layers, h, hv, hl, pos_tol=1e-3, field=w.field)
        assert bool(ok[s]) == r["ok"]
        if not r["ok"]:
            continue
        assert PT.par_ok(par[s], r["par"])[0], s
        assert PT.chi2_ok(chi2[s], r["chi2"]), (chi2[s], r["chi2"])
        worst = max(worst, PT.cov_err(mkf.unpack_cov(cov[s]), r["cov"]))
    say("seeds", b.seed_hits.shape[0], "worst covariance", worst)
    assert worst < PT.COV_REL_GRAZING


@pytest.mark.parametrize("flags", [0, 1])
def test_find_in_the_field_matches_oracle(mkf, flags):
    w = barrel_endcap_field()
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
        ref = O.find_event(w.find, w.layers, E, seeds=seeds, field=w.field)
        out = PT.compare_tracks(tr[pick], ref, mkf.unpack_cov)
        say({k: (v if k != "fail" else len(v)) for k, v in out.items()})
        assert not out["fail"], out["fail"][:5]
        assert out["equal"] >= 0.9 * out["n"]
        for k, (i, r) in enumerate(zip(pick, ref)):
            if not r["seed_ok"] or list(tr[i]["hit"][:len(r["plan"])]) != list(r["hit"]):
                continue
            st, p, Cm, c2, _ = O.backward_fit(w.find, w.layers, E, seeds[k], r,
                                              field=w.field)
            assert bf[3][i] == st
            if st == 1:
                assert PT.par_ok(bf[0][i], p)[0] and PT.chi2_ok(bf[2][i], c2), (i, bf[0][i], p)
                worst_bf = max(worst_bf, PT.cov_err(mkf.unpack_cov(bf[1][i]), Cm))
            h, hv, hl = seed_inputs(E, seeds[k])
            sd = O.seed(w.find, w.layers, h, hv, hl, field=w.field)
            m, _, sp, sc = O.smooth_track(w.find, w.layers, E, hl[2], sd["par"], sd["cov"], r,
                                          field=w.field)
            assert sm[2][i] == m
            for q in range(max(m, 0)):
                assert PT.par_ok(sm[0][i, q], sp[q])[0], (i, q)
                worst_sm = max(worst_sm, PT.cov_err(mkf.unpack_cov(sm[1][i, q]), sc[q]))
    say("worst covariance: backward fit", worst_bf, "smoothing", worst_sm)
    assert worst_bf < PT.COV_REL_GRAZING and worst_sm < PT.COV_REL_GRAZING


def test_cleared_field_gives_the_uniform_results(mkf):
    w = barrel_endcap_field()
    b = generate(w, events=[0])
    ref = context(mkf, w, b, field=False)
    ref.find()
    n = b.seed_hits.shape[0]
    a = ref.get_tracks(n)
    ref.close()
    ctx = context(mkf, w, b)
    ctx.find()
    with_field = ctx.get_tracks(n)
    ctx.load_field(None)
    ctx.seed(dev(b.seed_event), dev(b.seed_hits))
    ctx.find()
    c = ctx.get_tracks(n)
    ctx.close()
    assert a.tobytes() == c.tobytes()
    assert a.tobytes() != with_field.tobytes()


def test_bad_field_is_an_argument_error(mkf):
    from dataclasses import replace
    w = barrel_endcap_field()
    f = w.field
    ctx = mkf.Context(w.find)
    for bad in (replace(f, b0=0.0), replace(f, c_z2=float("inf")), replace(f, h_max=0.0),
                replace(f, h_max=1000.0)):
        with pytest.raises(mkf.MkfError) as ei:
            ctx.load_field(bad)
        assert ei.value.status == mkf.MKF_E_ARG
    ctx.close()


@pytest.fixture(scope="module")
def field_weights(mkf):
    """The surrogate trained on the field's own stepped crossings (its
    sampler propagates in the loaded field)."""
    w = barrel_endcap_field()
    ctx = mkf.Context(w.find)
    ctx.load_geometry(w.layers)
    ctx.load_field(w.field)
    rep = ctx.surrogate_train(n_samples=1 << 20, epochs=2, batch=512, lr=3e-3, seed=17,
                              loss_w=(1, .01, .01, .01, .01, .01, .01))
    say("field training", rep)
    p = ctx.surrogate_get()
    ctx.close()
    assert rep["loss_last"] < 0.05 * rep["loss_first"]
    return p


def test_field_surrogate_matches_oracle_and_the_stepped_search(mkf, field_weights):
    """In the solenoid-like field the surrogate form starts the barrel
    crossings from the network's path (equal steps to it, one Newton step
    as one more Runge-Kutta step).  With the field-trained weights most
    hints are kept and the hit lists are those of the full stepped search
    for at least 99.5% of seeds, with the oracle's tracks on sampled seeds;
    with large random weights every hint is refused and the tracks are bit
    for bit those of the form without the surrogate (zero weights would
    predict the straight line, which passes the check for stiff tracks)."""
    w = barrel_endcap_field()
    b = generate(w, events=[0, 1])
    n = b.seed_hits.shape[0]
    plain = context(mkf, w, b, mkf.F_BATCHED)
    plain.find()
    tp = plain.get_tracks(n)
    plain.close()
    garbage = (np.random.default_rng(95).normal(size=field_weights.size) * 8.0).astype(np.float32)
    for label, params in (("trained", field_weights), ("garbage", garbage)):
        ctx = mkf.Context(w.find, flags=mkf.F_BATCHED | mkf.F_SURROGATE)
        ctx.load_geometry(w.layers)
        ctx.load_field(w.field)
        ctx.surrogate_set(params)
        ctx.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v),
                      dev(b.layer))
        ctx.seed(dev(b.seed_event), dev(b.seed_hits))
        ctx.find()
        ts = ctx.get_tracks(n)
        st = ctx.stats()
        ctx.close()
        kept, rej = st["sur_kept"], st["sur_rejected"]
        same = np.all(ts["hit"] == tp["hit"], axis=1).mean()
        say(label, "kept", kept, "rejected", rej, "same hit lists", same)
        if label == "garbage":
            assert kept == 0 and rej > 0
            assert ts.tobytes() == tp.tobytes()
            continue
        assert kept >= 0.4 * (kept + rej)
        assert same >= 0.995
        rng = np.random.default_rng(94)
        for e in range(2):
            E = b.events[e]
            sel = np.nonzero(b.seed_event == e)[0]
            pick = np.sort(rng.choice(sel, 100, replace=False))
            ref = O.find_event(w.find, w.layers, E, seeds=E.seeds[pick - sel[0]],
                               field=w.field)
            out = PT.compare_tracks(ts[pick], ref, mkf.unpack_cov)
            say(e, {k: (v if k != "fail" else len(v)) for k, v in out.items()})
            assert not out["fail"], out["fail"][:5]
            assert out["equal"] >= 0.9 * out["n"]


def test_find_counters_agree_between_forms(mkf, field_weights):
    """mkf_stats' decision and work counters: both find forms evaluate the
    same candidates with the same arithmetic, so they count the same
    near-cut chi2 decisions, Runge-Kutta steps and Newton iterations; the
    uniform field takes no steps; every Newton iteration is one Runge-Kutta
    step.  The surrogate form's counts are reported beside them."""
    w = barrel_endcap_field()
    b = generate(w, events=[0, 1])
    rows = {}
    for field in (True, False):
        for flags in (0, mkf.F_BATCHED):
            ctx = context(mkf, w, b, flags, field=field)
            ctx.find()
            st = ctx.stats()
            ctx.close()
            rows[(field, flags)] = (st["n_near_cut"], st["n_rk_steps"], st["n_newton"])
            say("field" if field else "uniform", "batched" if flags else "plain",
                rows[(field, flags)], "steps", st["n_steps"])
    ctx = context(mkf, w, b, mkf.F_BATCHED | mkf.F_SURROGATE)
    ctx.surrogate_set(field_weights)
    ctx.find()
    st = ctx.stats()
    ctx.close()
    say("field surrogate", (st["n_near_cut"], st["n_rk_steps"], st["n_newton"]),
        "hints kept", st["sur_kept"], "rejected", st["sur_rejected"])
    assert rows[(True, 0)] == rows[(True, mkf.F_BATCHED)]
    assert rows[(False, 0)] == rows[(False, mkf.F_BATCHED)]
    nc, rk, nw = rows[(True, 0)]
    assert nc > 0 and rk > 0 and 0 < nw < rk
    assert rows[(False, 0)][0] > 0 and rows[(False, 0)][1:] == (0, 0)
    assert st["n_rk_steps"] > 0 and st["n_newton"] > 0
