"""GPU parity of the Rauch-Tung-Striebel smoothing of found tracks: the HIP
path through the C ABI (find, then mkf_smooth) against the oracle's smoother
of the oracle's own found tracks (from the oracle's seed fit), compared on
every surface for the seeds whose hit lists agree.  Needs an MI355X."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import barrel_endcap, generate, small_barrel
import parity as PT

pytestmark = pytest.mark.gpu

WORKERS = 8  # event generation processes (sized for a 16-CPU host)
NS = O.MAX_PLAN + 1

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


def find_and_smooth(M, w, b, flags=0):
    ctx = M.Context(w.find, flags=flags)
    ctx.load_geometry(w.layers)
    ctx.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v),
                  dev(b.layer))
    ctx.seed(dev(b.seed_event), dev(b.seed_hits))
    ctx.find()
    n = b.seed_hits.shape[0]
    tr = ctx.get_tracks(n)
    outs = [torch.zeros((n, NS, 6), device="cuda"), torch.zeros((n, NS, 21), device="cuda"),
            torch.full((n,), 99, dtype=torch.int32, device="cuda")]
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    ctx.smooth(*outs)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    ctx.close()
    return tr, [o.cpu().numpy() for o in outs], ms


def compare_smooth(M, w, ev, seeds, gtr, gsm, ref):
    """gtr: GPU track records of the seeds; gsm: (par, cov, n) rows of the
    same seeds; ref: the oracle's find results for them."""
    g_par, g_cov, g_n = gsm
    out = {"n": 0, "equal": 0, "surfaces": 0, "hits_differ": 0, "grazing": 0,
           "max_cov_err": 0.0, "max_cov_err_grazing": 0.0, "fail": []}
    for i, r in enumerate(ref):
        out["n"] += 1
        sh = seeds[i]
        if not r["seed_ok"]:
            if g_n[i] != 0:
                out["fail"].append((i, "n", int(g_n[i]), 0))
            continue
        n = len(r["plan"])
        if gtr[i]["plan_len"] != n or list(gtr[i]["hit"][:n]) != list(r["hit"]):
            out["hits_differ"] += 1
            continue
        h = np.array([[ev.x[j], ev.y[j], ev.z[j]] for j in sh], float).ravel()
        hv = np.array([[ev.var_u[j], ev.var_v[j]] for j in sh], float).ravel()
        sd = O.seed(w.find, w.layers, h, hv, [int(ev.layer[j]) for j in sh])
        m, lay, par, cov = O.smooth_track(w.find, w.layers, ev, int(ev.layer[sh[2]]), sd["par"],
                                          sd["cov"], r)
        if g_n[i] != m:
            out["fail"].append((i, "n", int(g_n[i]), m))
            continue
        hits = [x for x in r["hit"] if x >= 0] + list(sh)
        graze = PT.conditioning(w, ev, hits) < PT.GRAZING_COS
        out["grazing"] += graze
        good = True
        for k in range(m):
            ok_p, rel = PT.par_ok(g_par[i, k], par[k])
            ce = PT.cov_err(M.unpack_cov(g_cov[i, k]), cov[k])
            key = "max_cov_err_grazing" if graze else "max_cov_err"
            out[key] = max(out[key], ce)
            ok_v = ce <= (PT.COV_REL_GRAZING if graze else PT.COV_REL_FOUND)
            out["surfaces"] += 1
            if not (ok_p and ok_v):
                out["fail"].append((i, k, "numeric", ok_p, ce, rel.tolist()))
                good = False
                break
        out["equal"] += good
    say({k: (v if k != "fail" else len(v)) for k, v in out.items()})
    assert not out["fail"], out["fail"][:5]
    return out


def test_smooth_small_barrel_matches_oracle(mkf):
    """200 tracks, ten cylinders, no material: every track's eight surfaces
    compared; the last smoothed state is the find's own final state."""
    w = small_barrel()
    b = generate(w)
    tr, sm, ms = find_and_smooth(mkf, w, b)
    ev = b.events[0]
    ref = O.find_event(w.find, w.layers, ev)
    out = compare_smooth(mkf, w, ev, ev.seeds, tr, sm, ref)
    assert out["equal"] == 200 and out["surfaces"] == 1600
    last = sm[0][np.arange(200), sm[2] - 1]
    say("last smoothed state bitwise equal to the find's:", bool(np.array_equal(last, tr["par"])))
    assert np.allclose(last, tr["par"], rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("flags", [0, 1])
def test_smooth_realistic_events_match_oracle(mkf, flags):
    """Two events of 5,000 tracks (scattering, inefficiency, 30% noise),
    both find forms; the oracle recomputes 150 sampled seeds per event."""
    w = barrel_endcap()
    b = generate(w, events=[0, 1])
    tr, sm, ms = find_and_smooth(mkf, w, b, flags=flags)
    say("smooth ms", ms)
    rng = np.random.default_rng(33)
    for e in range(2):
        sel = np.nonzero(b.seed_event == e)[0]
        pick = np.sort(rng.choice(sel, 150, replace=False))
        seeds = b.events[e].seeds[pick - sel[0]]
        ref = O.find_event(w.find, w.layers, b.events[e], seeds=seeds)
        out = compare_smooth(mkf, w, b.events[e], seeds, tr[pick], [a[pick] for a in sm], ref)
        assert out["equal"] >= 0.9 * out["n"]


def test_smooth_full_workload_sampled(mkf):
    """The benchmark's workload (100 events x 5,000 tracks), one persistent
    find and one smoothing pass; the oracle recomputes 100 sampled seeds and
    every seed whose smoothing failed."""
    w = barrel_endcap()
    b = generate(w, workers=WORKERS)
    tr, sm, ms = find_and_smooth(mkf, w, b, flags=mkf.F_BATCHED)
    n = b.seed_hits.shape[0]
    ok = tr["status"] == 1
    say("smoothing of", n, "tracks:", ms, "ms; surfaces", int(sm[2][sm[2] > 0].sum()),
        "counts of n <= 0", np.unique(sm[2][sm[2] <= 0], return_counts=True))
    assert np.all(sm[2][~ok] == 0)
    assert np.mean(sm[2][ok] > 0) > 0.999
    rng = np.random.default_rng(34)
    failed = np.nonzero(ok & (sm[2] <= 0))[0]
    pick = np.union1d(np.sort(rng.choice(n, 100, replace=False)), failed)
    for e in np.unique(b.seed_event[pick]):
        sel = pick[b.seed_event[pick] == e]
        base = np.nonzero(b.seed_event == e)[0][0]
        seeds = b.events[e].seeds[sel - base]
        ref = O.find_event(w.find, w.layers, b.events[e], seeds=seeds)
        compare_smooth(mkf, w, b.events[e], seeds, tr[sel], [a[sel] for a in sm], ref)


def test_smooth_before_find_is_an_order_error(mkf):
    w = small_barrel()
    ctx = mkf.Context(w.find)
    ctx.load_geometry(w.layers)
    z = torch.zeros(6, device="cuda")
    with pytest.raises(mkf.MkfError) as ei:
        ctx.smooth(z, z, z)
    assert ei.value.status == mkf.MKF_E_ORDER
    ctx.close()
