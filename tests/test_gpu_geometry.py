"""GPU parity on the CMS-like geometry (stereo layers, a barrel gap, disk
rings without sensors): seeding, both find forms, backward fit and
smoothing against the oracle on the same events.  Needs an MI355X."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import cms_like, generate, make_batch, generate_event
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


def context(M, w, b, flags=0):
    ctx = M.Context(w.find, flags=flags)
    ctx.load_geometry(w.layers)
    ctx.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v),
                  dev(b.layer))
    ctx.seed(dev(b.seed_event), dev(b.seed_hits))
    return ctx


@pytest.mark.parametrize("flags", [0, 1])
def test_find_cms_like_matches_oracle(mkf, flags):
    w = cms_like()
    b = generate(w, events=[0, 1])
    ctx = context(mkf, w, b, flags)
    ctx.find()
    n = b.seed_hits.shape[0]
    tr = ctx.get_tracks(n)
    # backward fit and smoothing of the same tracks
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
    rng = np.random.default_rng(81)
    worst_bf = worst_sm = 0.0
    for e in range(2):
        E = b.events[e]
        sel = np.nonzero(b.seed_event == e)[0]
        pick = np.sort(rng.choice(sel, 120, replace=False))
        seeds = E.seeds[pick - sel[0]]
        ref = O.find_event(w.find, w.layers, E, seeds=seeds)
        out = PT.compare_tracks(tr[pick], ref, mkf.unpack_cov)
        say({k: (v if k != "fail" else len(v)) for k, v in out.items()})
        assert not out["fail"], out["fail"][:5]
        assert out["equal"] >= 0.9 * out["n"]
        for k, (i, r) in enumerate(zip(pick, ref)):
            if not r["seed_ok"]:
                continue
            nrm = len(r["plan"])
            if list(tr[i]["hit"][:nrm]) != list(r["hit"]):
                continue
            st, p, Cm, c2, nu = O.backward_fit(w.find, w.layers, E, seeds[k], r)
            assert bf[3][i] == st
            if st == 1:
                assert PT.par_ok(bf[0][i], p)[0] and PT.chi2_ok(bf[2][i], c2), (i, bf[0][i], p)
                worst_bf = max(worst_bf, PT.cov_err(mkf.unpack_cov(bf[1][i]), Cm))
            sh = seeds[k]
            h = np.array([[E.x[j], E.y[j], E.z[j]] for j in sh], float).ravel()
            hv = np.array([[E.var_u[j], E.var_v[j]] for j in sh], float).ravel()
            sd = O.seed(w.find, w.layers, h, hv, [int(E.layer[j]) for j in sh])
            m, _, sp, sc = O.smooth_track(w.find, w.layers, E, int(E.layer[sh[2]]), sd["par"],
                                          sd["cov"], r)
            assert sm[2][i] == m
            for q in range(max(m, 0)):
                assert PT.par_ok(sm[0][i, q], sp[q])[0], (i, q)
                worst_sm = max(worst_sm, PT.cov_err(mkf.unpack_cov(sm[1][i, q]), sc[q]))
    say("worst covariance: backward fit", worst_bf, "smoothing", worst_sm)
    assert worst_bf < PT.COV_REL_GRAZING and worst_sm < PT.COV_REL_GRAZING


def test_seed_states_cms_like_match_oracle(mkf):
    w = cms_like()
    ev = generate_event(w, 2, n_tracks=800)
    b = make_batch([ev])
    ctx = context(mkf, w, b)
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
        assert PT.par_ok(par[s], r["par"])[0], s
        if list(plan[s, :plen[s]]) != list(r["plan"]):
            assert r["plan_fragile"], (s, plan[s, :plen[s]], r["plan"])
            bad += 1
    assert bad <= 0.01 * b.seed_hits.shape[0] + 1


def test_bad_stereo_or_hole_is_a_geometry_error(mkf):
    from synth import Layer, FindConfig
    ctx = mkf.Context(FindConfig())
    for bad in (Layer(0, 10.0, -50, 50, 1e-5, 1e-4, stereo=2.0),
                Layer(0, 10.0, -50, 50, 1e-5, 1e-4, hole_lo=float("nan"), hole_hi=1.0)):
        with pytest.raises(mkf.MkfError) as ei:
            ctx.load_geometry([bad])
        assert ei.value.status == mkf.MKF_E_GEOMETRY
    ctx.close()
