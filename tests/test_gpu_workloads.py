"""GPU tests at full workload sizes: 512 events of uneven size in one
persistent graph launch (against the layer-synchronous form, against one
launch per event, and against the oracle on sampled seeds), dense events
with the surrogate, and a fit-only stress of 2 million tracks."""
import os
import time

import numpy as np
import pytest

from oracle import oracle as O
from synth import batched_uneven, dense, generate, make_batch
from synth.events import generate_event
from synth.fitstress import fit_stress
import parity as PT

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

WORKERS = max(1, min(16, os.cpu_count() or 1))


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def mkf():
    from paper_1811_04141_amd import mkf as M
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return M


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def find(M, w, b, flags, stream=None, autotune=False, params=None, repeats=1):
    ctx = M.Context(w.find, flags=flags, stream=stream)
    ctx.load_geometry(w.layers)
    if params is not None:
        ctx.surrogate_set(params)
    ctx.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v),
                  dev(b.layer))
    ctx.seed(dev(b.seed_event), dev(b.seed_hits))
    if autotune:
        ctx.autotune(repeats=1)
    for _ in range(repeats):
        ctx.find()
    tr = ctx.get_tracks(b.seed_hits.shape[0])
    st = ctx.stats()
    ctx.close()
    return tr, st


def without_seed_id(tr):
    t = tr.copy()
    t["seed_id"] = 0
    return t.tobytes()


def oracle_sample(M, w, b, picks):
    """Compare sampled seeds (global seed ids) with the oracle, event by event."""
    out_all = []
    for e in np.unique(b.seed_event[picks]):
        sel = np.nonzero(b.seed_event == e)[0]
        mine = np.sort(picks[b.seed_event[picks] == e])
        ref = O.find_event(w.find, w.layers, b.events[e], seeds=b.events[e].seeds[mine - sel[0]])
        out_all.append((e, mine, ref))
    return out_all


def test_uneven_512_events_one_launch(mkf):
    """512 events of 500-20,000 tracks (log-uniform) in one persistent,
    graph-replayed, autotuned launch, as the benchmark runs the find."""
    w = batched_uneven()
    t0 = time.time()
    b = generate(w, workers=WORKERS)
    n = b.seed_hits.shape[0]
    say(f"generated {w.name}: {b.x.shape[0]} hits, {n} seeds in {time.time() - t0:.1f}s")
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        tr, st = find(mkf, w, b, mkf.F_BATCHED | mkf.F_GRAPH, stream=stream.cuda_stream,
                      autotune=True, repeats=2)
    torch.cuda.synchronize()
    say("graph find ms", st["find_ms"], "steps", st["n_steps"])
    # the layer-synchronous form over the whole batch gives the same bytes
    tp, sp = find(mkf, w, b, 0)
    assert sp["n_steps"] == st["n_steps"]
    assert tp.tobytes() == tr.tobytes()
    # one launch per event (the plain comparison) for the smallest, the
    # largest and a middle event
    counts = np.bincount(b.seed_event, minlength=w.n_events)
    for e in [int(np.argmin(counts)), int(np.argmax(counts)), 257]:
        one = make_batch([b.events[e]])
        te, _ = find(mkf, w, one, 0)
        sel = np.nonzero(b.seed_event == e)[0]
        assert without_seed_id(te) == without_seed_id(tr[sel]), e
    # the oracle on sampled seeds of those and of random events
    rng = np.random.default_rng(12)
    picks = []
    for e in [int(np.argmin(counts)), int(np.argmax(counts))] + list(rng.choice(512, 2)):
        sel = np.nonzero(b.seed_event == e)[0]
        picks.append(rng.choice(sel, min(30, sel.size), replace=False))
    for e, mine, ref in oracle_sample(mkf, w, b, np.concatenate(picks)):
        out = PT.compare_tracks(tr[mine], ref, mkf.unpack_cov)
        say(e, {k: (v if k != "fail" else len(v)) for k, v in out.items()})
        assert not out["fail"], out["fail"][:5]
        assert out["tie_diverged"] + out["plan_diverged"] <= 0.05 * out["n"] + 1


def test_dense_events_surrogate_and_batching(mkf):
    """Two events of 25,000 tracks with 50% noise hits, found by the
    persistent graph form with the trained surrogate: the same hits as the
    plain find, and the oracle on sampled seeds."""
    w = dense(2)
    b = generate(w, workers=WORKERS)
    ctx = mkf.Context(w.find, flags=mkf.F_BATCHED)
    ctx.load_geometry(w.layers)
    rep = ctx.surrogate_train(n_samples=1 << 20, epochs=4, batch=512, lr=3e-3, seed=11,
                              loss_w=(1, .01, .01, .01, .01, .01, .01))
    params = ctx.surrogate_get()
    ctx.close()
    say("training", rep)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        ts, ss = find(mkf, w, b, mkf.F_BATCHED | mkf.F_GRAPH | mkf.F_SURROGATE,
                      stream=stream.cuda_stream, params=params, repeats=2)
    torch.cuda.synchronize()
    tp, sp = find(mkf, w, b, 0)
    kept, rej = ss["sur_kept"], ss["sur_rejected"]
    say("dense: steps", ss["n_steps"], "kept", kept, "rejected", rej)
    assert kept >= 0.5 * (kept + rej)
    assert np.array_equal(ts["status"], tp["status"])
    same = np.all(ts["hit"] == tp["hit"], axis=1)
    say("identical hit lists", same.mean())
    assert same.mean() >= 0.995
    rng = np.random.default_rng(13)
    picks = np.concatenate([rng.choice(np.nonzero(b.seed_event == e)[0], 50, replace=False)
                            for e in range(2)])
    for e, mine, ref in oracle_sample(mkf, w, b, picks):
        out = PT.compare_tracks(ts[mine], ref, mkf.unpack_cov)
        say(e, {k: (v if k != "fail" else len(v)) for k, v in out.items()})
        assert not out["fail"], out["fail"][:5]
        assert out["tie_diverged"] + out["plan_diverged"] <= 0.05 * out["n"] + 1


def test_fit_stress_two_million_tracks(mkf):
    """The fit alone over 2,000,000 tracks x 26 layers (random barrel or
    endcap geometry); sampled tracks against the oracle's fit."""
    n, k = 2_000_000, 26
    t0 = time.time()
    f = fit_stress(n, k, workers=WORKERS)
    say(f"generated fit stress {n} x {k} in {time.time() - t0:.1f}s")
    from synth import FindConfig
    fc = FindConfig()
    ctx = mkf.Context(fc)
    ins = [dev(a) for a in (f.kind, f.pos, f.x, f.y, f.z, f.var_u, f.var_v, f.length,
                             f.init_par, f.init_cov)]
    outs = [torch.zeros((n, 6), device="cuda"), torch.zeros((n, 21), device="cuda"),
            torch.zeros(n, device="cuda"), torch.zeros(n, dtype=torch.int32, device="cuda")]
    ctx.fit(*ins, *outs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.fit(*ins, *outs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    say(f"fit: {n * k / dt:.3e} track-layer updates/s ({dt * 1e3:.2f} ms)")
    g_par, g_cov, g_chi, g_st = (o.cpu().numpy() for o in outs)
    ctx.close()
    assert np.all(g_st == 0)
    worst = 0.0
    for t in np.random.default_rng(14).choice(n, 100, replace=False):
        rc, p, Cm, c2 = O.fit_track(fc, f.init_par[t].astype(float),
                                    mkf.unpack_cov(f.init_cov[t]).astype(float),
                                    f.kind[:, t].astype(np.int32), f.pos[:, t].astype(float),
                                    np.stack([f.x[:, t], f.y[:, t], f.z[:, t]], 1).astype(float),
                                    f.var_u[:, t].astype(float), f.var_v[:, t].astype(float))
        assert rc == 0
        ok, rel = PT.par_ok(g_par[t], p)
        assert ok, (t, rel)
        assert PT.chi2_ok(g_chi[t], c2), (t, g_chi[t], c2)
        worst = max(worst, PT.cov_err(mkf.unpack_cov(g_cov[t]), Cm))
    say("fit stress: worst covariance error (correlation units)", worst)
    assert worst <= PT.COV_REL_FOUND
