"""GPU parity of the backward fit of found tracks: the HIP path through the
C ABI (find, then mkf_backward_fit) against the oracle's backward fit of
the oracle's own found tracks, compared for the seeds whose hit lists agree.
Needs an MI355X."""
import time

import numpy as np
import pytest

from oracle import oracle as O
from synth import barrel_endcap, generate, small_barrel
import parity as PT

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


def find_and_backfit(M, w, b, flags=0):
    ctx = M.Context(w.find, flags=flags)
    ctx.load_geometry(w.layers)
    ctx.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v),
                  dev(b.layer))
    ctx.seed(dev(b.seed_event), dev(b.seed_hits))
    ctx.find()
    n = b.seed_hits.shape[0]
    tr = ctx.get_tracks(n)
    outs = [torch.full((n, 6), 7.0, device="cuda"), torch.full((n, 21), 7.0, device="cuda"),
            torch.full((n,), 7.0, device="cuda"), torch.full((n,), 7, dtype=torch.int32,
                                                            device="cuda")]
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    ctx.backward_fit(*outs)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    ctx.close()
    return tr, [o.cpu().numpy() for o in outs], ms


def compare_backfit(M, w, ev, seeds, gtr, gbf, ref):
    """gtr: GPU track records of the seeds; gbf: (par, cov, chi2, status)
    rows of the same seeds; ref: the oracle's find results for them."""
    g_par, g_cov, g_chi, g_st = gbf
    out = {"n": 0, "equal": 0, "hits_differ": 0, "grazing": 0, "max_cov_err": 0.0,
           "max_cov_err_grazing": 0.0, "fail": []}
    for i, r in enumerate(ref):
        out["n"] += 1
        st, p, Cm, c2, nu = O.backward_fit(w.find, w.layers, ev, seeds[i], r)
        if not r["seed_ok"]:
            if g_st[i] != 0 or np.any(g_par[i] != 0):
                out["fail"].append((i, "status", int(g_st[i]), st))
            continue
        n = len(r["plan"])
        if gtr[i]["plan_len"] != n or list(gtr[i]["hit"][:n]) != list(r["hit"]):
            out["hits_differ"] += 1
            continue
        if g_st[i] != st:
            out["fail"].append((i, "status", int(g_st[i]), st))
            continue
        if st != 1:
            continue
        assert nu == r["n_hits"]
        ok_p, rel = PT.par_ok(g_par[i], p)
        ok_c = PT.chi2_ok(g_chi[i], c2)
        ce = PT.cov_err(M.unpack_cov(g_cov[i]), Cm)
        hits = [h for h in r["hit"] if h >= 0] + list(seeds[i])
        graze = PT.conditioning(w, ev, hits) < PT.GRAZING_COS
        if graze:
            out["grazing"] += 1
            out["max_cov_err_grazing"] = max(out["max_cov_err_grazing"], ce)
            ok_v = ce <= PT.COV_REL_GRAZING
        else:
            out["max_cov_err"] = max(out["max_cov_err"], ce)
            ok_v = ce <= PT.COV_REL_FOUND
        if ok_p and ok_c and ok_v:
            out["equal"] += 1
        else:
            out["fail"].append((i, "numeric", ok_p, ok_c, ce, rel.tolist(), float(g_chi[i]), c2))
    say({k: (v if k != "fail" else len(v)) for k, v in out.items()})
    assert not out["fail"], out["fail"][:5]
    return out


def test_backward_fit_small_barrel_matches_oracle(mkf):
    """200 tracks, ten cylinders, no material: every track's ten hits are
    found on both sides, so every backward fit is compared."""
    w = small_barrel()
    b = generate(w)
    tr, bf, ms = find_and_backfit(mkf, w, b)
    ev = b.events[0]
    ref = O.find_event(w.find, w.layers, ev)
    out = compare_backfit(mkf, w, ev, ev.seeds, tr, bf, ref)
    assert out["equal"] == 200


@pytest.mark.parametrize("flags", [0, 1])
def test_backward_fit_realistic_events_match_oracle(mkf, flags):
    """Two events of 5,000 tracks (scattering, inefficiency, 30% noise),
    both find forms; the oracle recomputes 150 sampled seeds per event."""
    w = barrel_endcap()
    b = generate(w, events=[0, 1])
    tr, bf, ms = find_and_backfit(mkf, w, b, flags=flags)
    say("backward fit ms", ms)
    rng = np.random.default_rng(31)
    for e in range(2):
        sel = np.nonzero(b.seed_event == e)[0]
        pick = np.sort(rng.choice(sel, 150, replace=False))
        local = pick - sel[0]
        seeds = b.events[e].seeds[local]
        ref = O.find_event(w.find, w.layers, b.events[e], seeds=seeds)
        out = compare_backfit(mkf, w, b.events[e], seeds, tr[pick],
                              [a[pick] for a in bf], ref)
        assert out["equal"] >= 0.9 * out["n"]


def test_backward_fit_full_workload_sampled(mkf):
    """The benchmark's workload (100 events x 5,000 tracks) found in one
    persistent launch and fitted backwards in one launch; the oracle
    recomputes 100 sampled seeds and every seed whose backward fit failed
    (a track that no longer reaches an inner surface on the way back)."""
    w = barrel_endcap()
    b = generate(w, workers=WORKERS)
    tr, bf, ms = find_and_backfit(mkf, w, b, flags=mkf.F_BATCHED)
    n = b.seed_hits.shape[0]
    ok = tr["status"] == 1
    say("backward fit of", n, "tracks:", ms, "ms; status counts",
        np.unique(bf[3], return_counts=True))
    assert np.all(bf[3][~ok] == 0)
    assert np.mean(bf[3][ok] == 1) > 0.999
    assert np.all(np.isfinite(bf[0][bf[3] == 1]))
    # every failed backward fit, plus 100 sampled seeds, recomputed by the
    # oracle (a failure must be the oracle's too, at the same surface)
    rng = np.random.default_rng(32)
    failed = np.nonzero(ok & (bf[3] != 1))[0]
    pick = np.union1d(np.sort(rng.choice(n, 100, replace=False)), failed)
    for e in np.unique(b.seed_event[pick]):
        sel = pick[b.seed_event[pick] == e]
        base = np.nonzero(b.seed_event == e)[0][0]
        seeds = b.events[e].seeds[sel - base]
        ref = O.find_event(w.find, w.layers, b.events[e], seeds=seeds)
        compare_backfit(mkf, w, b.events[e], seeds, tr[sel], [a[sel] for a in bf], ref)


def test_backward_fit_before_find_is_an_order_error(mkf):
    w = small_barrel()
    ctx = mkf.Context(w.find)
    ctx.load_geometry(w.layers)
    z = torch.zeros(6, device="cuda")
    with pytest.raises(mkf.MkfError) as ei:
        ctx.backward_fit(z, z, z, z)
    assert ei.value.status == mkf.MKF_E_ORDER
    ctx.close()
