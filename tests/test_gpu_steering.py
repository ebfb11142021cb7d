"""GPU parity of region steering (mkf_load_steering): five eta regions on the
CMS-like geometry, seed plans, both find forms and the backward fit and
smoothing of the steered tracks against the oracle; host-side validation of
the region records.  Needs an MI355X."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import Region, cms_like, five_regions, generate
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


@pytest.fixture(scope="module")
def case():
    w = cms_like()
    return w, generate(w, events=[0, 1])


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def context(M, w, b, steering, flags=0):
    ctx = M.Context(w.find, flags=flags)
    ctx.load_geometry(w.layers)
    if steering is not None:
        ctx.load_steering(steering)
    ctx.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v),
                  dev(b.layer))
    ctx.seed(dev(b.seed_event), dev(b.seed_hits))
    return ctx


def seed_inputs(E, sh):
    h = np.array([[E.x[j], E.y[j], E.z[j]] for j in sh], float).ravel()
    hv = np.array([[E.var_u[j], E.var_v[j]] for j in sh], float).ravel()
    return h, hv, [int(E.layer[j]) for j in sh]


def test_steered_plans_match_oracle(mkf, case):
    w, b = case
    st = five_regions()
    ctx = context(mkf, w, b, st)
    _, _, ok, plen, plan, _ = ctx.get_seed_states(b.seed_hits.shape[0])
    # an empty steering returns to the helix plans
    ctx.load_steering([])
    ctx.seed(dev(b.seed_event), dev(b.seed_hits))
    _, _, ok2, plen2, plan2, _ = ctx.get_seed_states(b.seed_hits.shape[0])
    ctx.close()
    assert np.array_equal(ok, ok2)
    n = bad = differ = 0
    for s in range(b.seed_hits.shape[0]):
        if not ok[s]:
            continue
        E = b.events[b.seed_event[s]]
        h, hv, hl = seed_inputs(E, b.seed_hits[s])
        r = O.seed(w.find, w.layers, h, hv, hl, steering=st)
        n += 1
        if list(plan[s, :plen[s]]) != list(r["plan"]):
            assert r["plan_fragile"], (s, plan[s, :plen[s]], r["plan"])
            bad += 1
        differ += list(plan[s, :plen[s]]) != list(plan2[s, :plen2[s]])
    say("seeds", n, "fragile differences", bad, "plans changed by steering", differ)
    assert n > 3000 and bad <= 0.001 * n + 1 and differ > 0.5 * n


@pytest.mark.parametrize("flags", [0, 1])
def test_steered_find_matches_oracle(mkf, case, flags):
    w, b = case
    st = five_regions()
    ctx = context(mkf, w, b, st, flags)
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
    rng = np.random.default_rng(91)
    worst_bf = worst_sm = 0.0
    for e in range(2):
        E = b.events[e]
        sel = np.nonzero(b.seed_event == e)[0]
        pick = np.sort(rng.choice(sel, 120, replace=False))
        seeds = E.seeds[pick - sel[0]]
        ref = O.find_event(w.find, w.layers, E, seeds=seeds, steering=st)
        out = PT.compare_tracks(tr[pick], ref, mkf.unpack_cov)
        say({k: (v if k != "fail" else len(v)) for k, v in out.items()})
        assert not out["fail"], out["fail"][:5]
        assert out["equal"] >= 0.9 * out["n"]
        for k, (i, r) in enumerate(zip(pick, ref)):
            if not r["seed_ok"] or list(tr[i]["hit"][:len(r["plan"])]) != list(r["hit"]):
                continue
            stt, p, Cm, c2, _ = O.backward_fit(w.find, w.layers, E, seeds[k], r)
            assert bf[3][i] == stt
            if stt == 1:
                assert PT.par_ok(bf[0][i], p)[0] and PT.chi2_ok(bf[2][i], c2), (i, bf[0][i], p)
                worst_bf = max(worst_bf, PT.cov_err(mkf.unpack_cov(bf[1][i]), Cm))
            h, hv, hl = seed_inputs(E, seeds[k])
            sd = O.seed(w.find, w.layers, h, hv, hl)
            m, _, sp, sc = O.smooth_track(w.find, w.layers, E, hl[2], sd["par"], sd["cov"], r)
            assert sm[2][i] == m
            for q in range(max(m, 0)):
                assert PT.par_ok(sm[0][i, q], sp[q])[0], (i, q)
                worst_sm = max(worst_sm, PT.cov_err(mkf.unpack_cov(sm[1][i, q]), sc[q]))
    say("worst covariance: backward fit", worst_bf, "smoothing", worst_sm)
    assert worst_bf < PT.COV_REL_GRAZING and worst_sm < PT.COV_REL_GRAZING


def test_bad_regions_are_argument_errors(mkf):
    w = cms_like()
    ctx = mkf.Context(w.find)
    with pytest.raises(mkf.MkfError) as ei:
        ctx.load_steering(five_regions())
    assert ei.value.status == mkf.MKF_E_ORDER
    ctx.load_geometry(w.layers)
    bad = ([Region(0.0, 1.0, (3, 28))],               # no layer 28
           [Region(0.0, 1.0, (3, 4, 3))],              # listed twice
           [Region(1.0, 1.0, (3,))],                   # empty range
           [Region(float("nan"), 1.0, (3,))],
           [Region(0.0, 1.0, (3,))] * 9)               # too many regions
    for st in bad:
        with pytest.raises(mkf.MkfError) as ei:
            ctx.load_steering(st)
        assert ei.value.status == mkf.MKF_E_ARG
    ctx.load_steering(five_regions())
    ctx.close()
