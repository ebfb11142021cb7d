"""Throughput of the Kalman-filter track finding hot path on one MI355X.

A step is one pass of the find (propagate, hit search, chi2, per-seed
selection, Kalman update over every plan layer of every seed) over the whole
workload: 512 synthetic barrel+endcap events of uneven size, 500-20,000
tracks each (log-uniform; scattering, 2% inefficiency, 30% noise hits), in
one persistent launch captured as a HIP graph, with the learned propagation
surrogate (trained on 10 M propagations before the timed region).  Beside it
the same events are found without the surrogate, in the layer-synchronous
form over all events, and one launch sequence per event (the plain
comparison).  Hits are indexed and seeds fitted before the timed region (the
paper times core finding without this pre-processing, Section 4.1); inputs
are resident in HBM.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K]
[--warmup W].
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "candidate-layer updates/s (propagate+chi2+update), surrogate+batched vs plain, 1 GPU"
UNIT = "candidate-layer updates/s"
FIT_TRACKS = 2_000_000  # the fit stress workload: 2 M tracks x 26 layers
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0
# Algorithmic cost of one candidate-layer step (counted from the kernel's
# arithmetic; see the design notes): FP32 flops and the bytes the
# layer-synchronous form must move through HBM.
FLOPS_PER_STEP = 780.0
PLAIN_BYTES_PER_STEP = 256.0
# fit: one track-layer update (crossing, transport, Jacobian, covariance,
# scattering, chi2, Kalman update) = the step count above without the window
FIT_FLOPS_PER_UPDATE = 727.0
# smoothing, per surface of a found track: the forward pass writes 91 words
# (filtered and predicted state, F C, layer), the backward pass reads them
# and writes the 27-word smoothed state (inputs not counted)
SMOOTH_BYTES_PER_SURFACE = 4.0 * (91 + 91 + 27)
# surrogate network per sample: forward 2 (8*64 + 64*64 + 7*64) = 10,112;
# backward (input errors of layers 3 and 2, weight gradients of all three)
# 19,200
MLP_FWD_FLOPS = 10112.0
MLP_FWD_BWD_FLOPS = 29312.0
# the surrogate's training (the uniform-field network of the find)
TRAIN = dict(n_samples=10_000_000, epochs=2, batch=512, lr=3e-3, seed=11,
             loss_w=(1, .01, .01, .01, .01, .01, .01))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def profiled_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter record
    (FETCH_SIZE and WRITE_SIZE, scaled by a 1 GiB copy), or None if the
    kernel sources changed since the counters were taken."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")):
        rec = json.load(open(path))
        if rec["kernel"] != kernel or rec["workload"] != workload:
            continue
        h = hashlib.sha256()
        for f in rec["sources"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() == rec["source_sha256"]:
            return rec["hbm_bytes_per_launch"]
    return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_share(job):
    """One worker of the CPU baseline: the oracle's find over the first seeds
    of one event, 50 at a time, until the time budget is spent."""
    w, ev, seconds = job
    from oracle import oracle as O
    n_done, steps, t_cpu = 0, 0, 0.0
    while t_cpu < seconds and n_done < ev.seeds.shape[0]:
        chunk = ev.seeds[n_done:n_done + 50]
        t1 = time.perf_counter()
        res = O.find_event(w.find, w.layers, ev, seeds=chunk)
        t_cpu += time.perf_counter() - t1
        steps += sum(r["n_steps"] for r in res)
        n_done += chunk.shape[0]
    return steps, t_cpu, n_done


def cpu_baseline(w, batch, seconds, workers):
    """The FP64 oracle as it stands on this machine's host CPUs: one thread
    on event 0, then one event per process on events 0..workers-1 (the
    paper's events-in-flight pattern, Section 4.2), each on the first seeds
    of its event for `seconds`; throughput is the summed steps over the
    longest worker's time."""
    one = _oracle_share((w, batch.events[0], seconds))
    n = max(1, min(workers, len(batch.events)))
    jobs = [(w, batch.events[e], seconds) for e in range(n)]
    if n == 1:
        out = [one]
    else:
        import multiprocessing as mp
        pool = mp.get_context("spawn").Pool(n)
        try:
            out = pool.map(_oracle_share, jobs, chunksize=1)
        finally:
            pool.close()  # the workers exit on their own
            pool.join()
    steps = sum(o[0] for o in out)
    t = max(o[1] for o in out)
    seeds = sum(o[2] for o in out)
    # one thread on the other workloads' shapes: the 200-track barrel event
    # (whole) and a dense 25,000-track event with 50% noise (first seeds)
    from synth import dense, generate_event, small_barrel
    others = {}
    for wo in (small_barrel(), dense(1)):
        so, to, no = _oracle_share((wo, generate_event(wo, 0), min(seconds, 3.0)))
        others[wo.name] = {"value": so / to, "seeds": no, "steps": so, "seconds": round(to, 2)}
    return {"value": steps / t, "unit": UNIT, "cores": n, "kind": "oracle",
            "sample": f"first seeds of events 0-{n - 1} of the workload, one event per process "
                      f"({seeds} seeds, {steps} candidate-layer steps, {t:.1f} s; FP64, "
                      f"brute-force hit scan)",
            "one_thread": {"value": one[0] / one[1], "sample":
                           f"first {one[2]} seeds of event 0 ({one[0]} steps, {one[1]:.1f} s)"},
            "other_workloads_one_thread": others,
            "cpu_model": cpu_model(), "hardware_concurrency": os.cpu_count(),
            "cpus_available": len(os.sched_getaffinity(0))}


def time_form(mkf, w, b, flags, stream, args, T, params=None, autotune=True):
    """One context of the given flags over the whole workload: warm-up, then
    K finds between device synchronisations.  Returns (result, tracks)."""
    import numpy as np
    import torch
    with torch.cuda.stream(stream):
        ctx = mkf.Context(w.find, flags=flags, stream=stream.cuda_stream)
        ctx.load_geometry(w.layers)
        if params is not None:
            ctx.surrogate_set(params)
        ctx.load_hits(b.ev_off, *[T(a) for a in (b.x, b.y, b.z, b.var_u, b.var_v, b.layer)])
        ctx.seed(T(b.seed_event), T(b.seed_hits))
        tuning = ctx.autotune(repeats=2) if (flags & mkf.F_BATCHED) and autotune else None
        for _ in range(args.warmup):
            ctx.find()
        torch.cuda.synchronize()
        find_ms, main_ms = [], []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.find()
            st = ctx.stats()
            find_ms.append(st["find_ms"])
            main_ms.append(st["main_ms"])
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        tr = ctx.get_tracks(b.seed_hits.shape[0])
        st = ctx.stats()
        ctx.close()
    res = {"ms_per_step": wall * 1e3, "find_ms": float(np.median(find_ms)),
           "main_ms": float(np.median(main_ms)), "main_launches": st["main_launches"],
           "n_steps": st["n_steps"], "value": st["n_steps"] / wall,
           "device_value": st["n_steps"] / (float(np.median(find_ms)) * 1e-3),
           "tuning": tuning}
    if flags & mkf.F_SURROGATE:
        res["surrogate"] = {"kept": st["sur_kept"], "rejected": st["sur_rejected"],
                            "kept_frac": st["sur_kept"] / max(1, st["sur_kept"] + st["sur_rejected"])}
    return res, tr


def time_per_event(mkf, w, b, stream, args, T):
    """The plain comparison: one context per event, each found by its own
    layer-synchronous launch sequence; a step finds every event once.  The
    find call returns after its event's work, so `value` counts the host's
    waits between events too; `device_value` sums the finds' device times."""
    import numpy as np
    import torch
    from synth import make_batch
    ctxs = []
    with torch.cuda.stream(stream):
        for e in range(w.n_events):
            one = make_batch([b.events[e]])
            c = mkf.Context(w.find, flags=0, stream=stream.cuda_stream)
            c.load_geometry(w.layers)
            c.load_hits(one.ev_off, *[T(a) for a in (one.x, one.y, one.z, one.var_u,
                                                    one.var_v, one.layer)])
            c.seed(T(one.seed_event), T(one.seed_hits))
            ctxs.append((c, one.seed_hits.shape[0]))
        for _ in range(args.warmup):
            for c, _ in ctxs:
                c.find()
        torch.cuda.synchronize()
        dev_ms = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            tot = 0.0
            for c, _ in ctxs:
                c.find()
                tot += c.stats()["find_ms"]
            dev_ms.append(tot)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        steps = sum(c.stats()["n_steps"] for c, _ in ctxs)
        launches = sum(c.stats()["n_launches"] for c, _ in ctxs)
        tr = np.concatenate([c.get_tracks(n) for c, n in ctxs])
        for c, _ in ctxs:
            c.close()
    off = np.concatenate([[0], np.cumsum([n for _, n in ctxs])[:-1]])
    tr["seed_id"] += np.repeat(off, [n for _, n in ctxs]).astype(np.int32)
    return ({"ms_per_step": wall * 1e3, "find_ms": float(np.median(dev_ms)), "n_steps": steps,
             "launches_per_step": launches, "value": steps / wall,
             "device_value": steps / (float(np.median(dev_ms)) * 1e-3)}, tr)


def measure_kernels(mkf, w, stream, T, f, batch, extended, params, gen_workers):
    """Throughput of the other hot-path kernels, each from HIP events on the
    context stream around one launch after a warm-up: the search-free fit
    (2 M tracks x 26 layers), the backward fit and the smoothing of the
    workload's found tracks, the surrogate network's inference and gradient
    (2^20 samples from its training sampler), and the find on dense events
    (4 x 25,000 tracks, 50% noise) with and without the surrogate (its
    weights: params, trained on the same geometry).  With `extended`:
    triplet seeding with cleaning, find and duplicate removal, the find with
    a material map and with region steering."""
    import numpy as np
    import torch

    def timed(fn):
        fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1)

    def alu(flops, ms, peak, unit_count, unit):
        ach = flops / (ms * 1e-3) / 1e12
        return {"ms": ms, "throughput": unit_count / (ms * 1e-3), "unit": unit,
                "achieved_tflops": ach, "peak_tflops": peak, "frac": ach / peak}

    hits = [T(a) for a in (batch.x, batch.y, batch.z, batch.var_u, batch.var_v, batch.layer)]
    seeds = (T(batch.seed_event), T(batch.seed_hits))
    out = {}
    with torch.cuda.stream(stream):
        ctx = mkf.Context(w.find, stream=stream.cuda_stream)
        ctx.load_geometry(w.layers)
        k, n = f.x.shape
        ins = [T(a) for a in (f.kind, f.pos, f.x, f.y, f.z, f.var_u, f.var_v, f.length,
                              f.init_par, f.init_cov)]
        dev = ins[0].device
        outs = [torch.zeros((n, 6), device=dev), torch.zeros((n, 21), device=dev),
                torch.zeros(n, device=dev), torch.zeros(n, dtype=torch.int32, device=dev)]
        ms = timed(lambda: ctx.fit(*ins, *outs))
        out["k_fit"] = dict(alu(FIT_FLOPS_PER_UPDATE * n * k, ms, FP32_VECTOR_PEAK_TFLOPS, n * k,
                                "track-layer updates/s"), bound="alu",
                            workload=f"{n} tracks x {k} layers")
        del ins, outs
        # backward fit of the tracks found in the workload, counted by its
        # updates (one per hit, the seed hits included; the propagations
        # through layers without a hit are not counted)
        ctx2 = mkf.Context(w.find, flags=mkf.F_BATCHED, stream=stream.cuda_stream)
        ctx2.load_geometry(w.layers)
        ctx2.load_hits(batch.ev_off, *hits)
        ctx2.seed(*seeds)
        ctx2.find()
        ns = batch.seed_hits.shape[0]
        tr = ctx2.get_tracks(ns)
        bouts = [torch.zeros((ns, 6), device=dev), torch.zeros((ns, 21), device=dev),
                 torch.zeros(ns, device=dev), torch.zeros(ns, dtype=torch.int32, device=dev)]
        ms = timed(lambda: ctx2.backward_fit(*bouts))
        ok = bouts[3].cpu().numpy() == 1
        upd = int(tr["n_hits"][ok].sum())
        out["k_backfit"] = dict(alu(FIT_FLOPS_PER_UPDATE * upd, ms, FP32_VECTOR_PEAK_TFLOPS, upd,
                                    "track-hit updates/s"), bound="alu",
                                workload=f"{int(ok.sum())} found tracks, {upd} hits")
        del bouts
        sm = [torch.zeros((ns, 33, 6), device=dev), torch.zeros((ns, 33, 21), device=dev),
              torch.zeros(ns, dtype=torch.int32, device=dev)]
        ms = timed(lambda: ctx2.smooth(*sm))
        nsurf = int(sm[2].clamp(min=0).sum().item())
        gbs = SMOOTH_BYTES_PER_SURFACE * nsurf / (ms * 1e-3) / 1e9
        out["k_smooth_fwd+bwd"] = {"ms": ms, "throughput": nsurf / (ms * 1e-3),
                                   "unit": "track-surface states/s", "achieved_gbs": gbs,
                                   "peak_gbs": HBM_PEAK_GBS, "frac": gbs / HBM_PEAK_GBS,
                                   "bound": "hbm",
                                   "workload": f"{int((sm[2] > 0).sum().item())} found tracks, "
                                               f"{nsurf} surfaces"}
        del sm
        ctx2.close()
        torch.cuda.empty_cache()
        m = 1 << 20
        x = torch.zeros((m, 8), device=dev)
        t = torch.zeros((m, 7), device=dev)
        v = torch.zeros(m, device=dev)
        ctx.surrogate_samples(m, 5, x, t, v)
        y = torch.zeros((m, 7), device=dev)
        ms = timed(lambda: ctx.surrogate_infer(x, y))
        out["k_mlp_infer"] = dict(alu(MLP_FWD_FLOPS * m, ms, BF16_MFMA_PEAK_TFLOPS, m,
                                      "samples/s"), bound="mfma", workload=f"{m} samples")
        lw = np.ones(7, np.float32)
        ms = timed(lambda: ctx.surrogate_grad(x, t, lw))
        out["k_mlp_grad+reduce"] = dict(alu(MLP_FWD_BWD_FLOPS * m, ms, BF16_MFMA_PEAK_TFLOPS, m,
                                            "samples/s"), bound="mfma", workload=f"{m} samples")
        del x, t, v, y
        ctx.close()
        torch.cuda.empty_cache()
        out["find_dense"] = measure_dense(mkf, stream, T, params, gen_workers)
        if extended:
            out.update(measure_extended(mkf, w, stream, T, batch, hits, seeds, timed))
    log("kernels", json.dumps(out))
    return out


def measure_extended(mkf, w, stream, T, batch, hits, seeds, timed):
    """The extended finds: triplet seeding, cleaning and duplicate removal;
    the find with a material map and with five-region steering."""
    import torch
    from synth import CleaningConfig, SeedingConfig, five_regions, material_map
    out = {}
    dev = hits[0].device
    ctx3 = mkf.Context(w.find, flags=mkf.F_BATCHED, stream=stream.cuda_stream)
    ctx3.load_geometry(w.layers)
    ctx3.load_hits(batch.ev_off, *hits)
    cap = 48 << 20
    sev = torch.zeros(cap, dtype=torch.int32, device=dev)
    shit = torch.zeros((cap, 3), dtype=torch.int32, device=dev)
    nt = [0]

    def mk():
        nt[0] = ctx3.make_seeds(SeedingConfig(), cap, sev, shit)

    ms_seed = timed(mk)
    ctx3.seed(sev[:nt[0]], shit[:nt[0]])
    keep = torch.zeros(nt[0], dtype=torch.int32, device=dev)
    nk = [0]

    def cl():
        nk[0] = ctx3.clean_seeds(CleaningConfig(), keep)

    ms_clean = timed(cl)
    ctx3.find()
    ctx3.find()
    find_ms = ctx3.stats()["find_ms"]
    dup = torch.zeros(nt[0], dtype=torch.int32, device=dev)
    nd = [0]

    def dd():
        nd[0] = ctx3.find_duplicates(0.5, dup)

    ms_dup = timed(dd)
    out["triplet_seeding_pipeline"] = {
        "workload": f"{w.name}, seeds from every triplet of layers 0-2",
        "triplets": nt[0], "make_seeds_ms": ms_seed, "clean_seeds_ms": ms_clean,
        "kept_after_cleaning": nk[0], "find_ms_all_triplet_seeds": find_ms,
        "duplicates": nd[0], "find_duplicates_ms": ms_dup}
    del sev, shit, keep, dup
    ctx3.close()
    variants = (("find_material_map",
                 lambda c: c.load_material(material_map(120.0, 300.0, 24, 30, 0.015, 0.1))),
                ("find_five_region_steering", lambda c: c.load_steering(five_regions())))
    for label, setup in variants:
        c4 = mkf.Context(w.find, flags=mkf.F_BATCHED, stream=stream.cuda_stream)
        c4.load_geometry(w.layers)
        setup(c4)
        c4.load_hits(batch.ev_off, *hits)
        c4.seed(*seeds)
        tun4 = c4.autotune(repeats=2)
        c4.find()
        c4.find()
        st = c4.stats()
        c4.close()
        out[label] = {"find_ms": st["find_ms"], "n_steps": st["n_steps"],
                      "throughput": st["n_steps"] / (st["find_ms"] * 1e-3),
                      "unit": UNIT, "workload": w.name, "tuning": tun4}
    return out


def measure_dense(mkf, stream, T, params, gen_workers, repeats=5):
    """The find on dense events (4 x 25,000 tracks, 50% noise hits), in the
    persistent form with and without the surrogate: median device time of
    `repeats` finds after autotuning, and the fraction of identical hit
    lists."""
    import numpy as np
    from synth import dense, generate
    wd = dense(4)
    bd = generate(wd, workers=gen_workers)
    hits = [T(a) for a in (bd.x, bd.y, bd.z, bd.var_u, bd.var_v, bd.layer)]
    seeds = (T(bd.seed_event), T(bd.seed_hits))
    n = int(bd.seed_hits.shape[0])
    out = {"workload": wd.name, "seeds": n, "hits": int(bd.x.shape[0])}
    tracks = {}
    forms = [("batched", mkf.F_BATCHED)]
    if params is not None:
        forms.append(("surrogate", mkf.F_BATCHED | mkf.F_SURROGATE))
    for label, flags in forms:
        c = mkf.Context(wd.find, flags=flags, stream=stream.cuda_stream)
        c.load_geometry(wd.layers)
        if label == "surrogate":
            c.surrogate_set(params)
        c.load_hits(bd.ev_off, *hits)
        c.seed(*seeds)
        tun = c.autotune(repeats=2)
        ms = []
        for _ in range(repeats):
            c.find()
            st = c.stats()
            ms.append(st["find_ms"])
        tracks[label] = c.get_tracks(n)
        c.close()
        f_ms = float(np.median(ms))
        out[label] = {"find_ms": f_ms, "n_steps": st["n_steps"],
                      "throughput": st["n_steps"] / (f_ms * 1e-3), "unit": UNIT, "tuning": tun,
                      "near_cut_decisions": st["n_near_cut"]}
        if label == "surrogate":
            out[label]["kept_fraction"] = st["sur_kept"] / max(1, st["sur_kept"] + st["sur_rejected"])
    if "surrogate" in tracks:
        out["same_hits"] = float(np.mean(np.all(tracks["surrogate"]["hit"] ==
                                                tracks["batched"]["hit"], axis=1)))
    return out


def validation(batch, tracks, plen, plan, ok):
    """Hit-selection accuracy and efficiency of found tracks against the
    generator's truth.  Accuracy: over the plan layers of every seed whose
    fit succeeded, the fraction where the selected hit is the seed's truth
    track's hit on that layer (a layer where the truth track left no hit
    counts as correct).  Efficiency: the fraction of those seeds whose track
    (its three seed hits and the found ones) has at least 75% hits of the
    seed's truth track.  Purity: found hits from the seed's truth track over
    all found hits."""
    import numpy as np
    evs = batch.events
    truth = np.concatenate([e.track for e in evs]).astype(np.int64)
    layer = np.asarray(batch.layer, np.int64)
    nl = int(layer.max()) + 1 if layer.size else 1
    ntrk = max(int(truth.max()) + 1, 1)
    ev_of_hit = np.repeat(np.arange(len(evs), dtype=np.int64), np.diff(batch.ev_off))
    real = truth >= 0
    keys = ((ev_of_hit[real] * ntrk + truth[real]) * nl + layer[real])
    gidx = np.nonzero(real)[0]
    order = np.argsort(keys, kind="stable")
    keys, gidx = keys[order], gidx[order]
    seed_track = np.concatenate([e.seed_track for e in evs]).astype(np.int64)
    sev = np.asarray(batch.seed_event, np.int64)
    base = batch.ev_off[sev]
    sel = np.asarray(tracks["hit"], np.int64)
    m = sel.shape[1]
    steps = np.arange(m)[None, :]
    valid = (steps < plen[:, None]) & (ok[:, None] != 0)
    qkey = ((sev * ntrk + seed_track)[:, None] * nl + plan[:, :m].astype(np.int64))
    pos = np.searchsorted(keys, qkey)
    posc = np.minimum(pos, max(keys.size - 1, 0))
    has_truth = (keys.size > 0) & (keys[posc] == qkey)
    truth_hit = np.where(has_truth, gidx[posc], -1)
    sel_g = np.where(sel >= 0, sel + base[:, None], -1)
    correct = (~has_truth) | (sel_g == truth_hit)
    found = (sel >= 0) & valid
    match = found & (truth[np.maximum(sel_g, 0)] == seed_track[:, None])
    n_found = found.sum(axis=1)
    n_match = match.sum(axis=1)
    good = ok != 0
    eff = ((3 + n_match) >= 0.75 * (3 + n_found)) & good
    return {"seeds": int(good.sum()),
            "hit_selection_accuracy": float(correct[valid].mean()) if valid.any() else None,
            "efficiency_75pct": float(eff.sum() / max(1, good.sum())),
            "hit_purity": float(n_match[good].sum() / max(1, n_found[good].sum())),
            "found_hits_per_track": float(n_found[good].mean()) if good.any() else None}


FIELD_TRAIN = dict(n_samples=10_000_000, epochs=2, batch=512, lr=3e-3, seed=17,
                   loss_w=(1, .01, .01, .01, .01, .01, .01))


def measure_field(mkf, stream, T, n_events, gen_workers, repeats=5):
    """The find in the parameterised solenoid-like field, on events of the
    barrel + endcap workload simulated in it (n_events x 5,000 tracks), with
    and without the learned surrogate.  Without it every barrel crossing is
    found by Runge-Kutta stepping and Newton iteration; with it the crossing
    starts from the network's path (equal steps to it and one Newton step,
    kept under the same checks, else the full stepped search).  The network
    is trained on 10 M stepped crossings of the field's own sampler.  Each
    form is autotuned, then timed as the median device time of `repeats`
    finds; the hit lists of the two forms are compared track by track."""
    import numpy as np
    import torch
    from synth import barrel_endcap_field, generate
    wf = barrel_endcap_field(n_events, 5000)
    t0 = time.time()
    bf = generate(wf, workers=gen_workers)
    log(f"{wf.name}: {bf.x.shape[0]} hits, {bf.seed_hits.shape[0]} seeds in "
        f"{time.time() - t0:.1f}s")
    fh = [T(a) for a in (bf.x, bf.y, bf.z, bf.var_u, bf.var_v, bf.layer)]
    fs = (T(bf.seed_event), T(bf.seed_hits))
    n = int(bf.seed_hits.shape[0])
    out = {"workload": wf.name, "events": n_events, "seeds": n}
    tracks = {}
    with torch.cuda.stream(stream):
        for label, flags in (("stepped", mkf.F_BATCHED),
                             ("surrogate", mkf.F_BATCHED | mkf.F_SURROGATE)):
            c = mkf.Context(wf.find, flags=flags, stream=stream.cuda_stream)
            c.load_geometry(wf.layers)
            c.load_field(wf.field)
            if label == "surrogate":
                out["training"] = c.surrogate_train(**FIELD_TRAIN)
                log("field surrogate trained", json.dumps(out["training"]))
            c.load_hits(bf.ev_off, *fh)
            c.seed(*fs)
            tun = c.autotune(repeats=2)
            ms, main = [], []
            for _ in range(repeats):
                c.find()
                st = c.stats()
                ms.append(st["find_ms"])
                main.append(st["main_ms"])
            tracks[label] = c.get_tracks(n)
            c.close()
            f_ms = float(np.median(ms))
            res = {"find_ms": f_ms, "main_ms": float(np.median(main)), "n_steps": st["n_steps"],
                   "throughput": st["n_steps"] / (f_ms * 1e-3), "unit": UNIT, "tuning": tun,
                   "rk_steps": st["n_rk_steps"], "newton_iterations": st["n_newton"],
                   "near_cut_decisions": st["n_near_cut"]}
            if label == "surrogate":
                kept, rej = st["sur_kept"], st["sur_rejected"]
                res["hints_kept"] = kept
                res["hints_rejected"] = rej
                res["kept_fraction"] = kept / max(1, kept + rej)
            out[label] = res
            log("field", label, json.dumps(res))
    out["same_hits"] = float(np.mean(np.all(tracks["surrogate"]["hit"] ==
                                            tracks["stepped"]["hit"], axis=1)))
    out["speedup"] = out["stepped"]["find_ms"] / out["surrogate"]["find_ms"]
    return out


FORMS = ("surrogate", "surrogate_eager", "graph", "batched", "plain_all_events",
         "plain_per_event")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=512)
    ap.add_argument("--forms", default=",".join(FORMS))
    ap.add_argument("--gen-workers", type=int, default=min(16, len(os.sched_getaffinity(0))),
                    help="host processes generating the events (1 under a profiler)")
    ap.add_argument("--workload-cache", default=None,
                    help="file holding the generated events: read if present, else written "
                         "(lets profiled runs skip the generation)")
    ap.add_argument("--surrogate-params", default=None,
                    help="file of the trained surrogate weights (.npy): read if present, else "
                         "written after training (lets profiled runs skip the training)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="budget of each leg of the oracle CPU baseline (0 disables)")
    ap.add_argument("--cpu-workers", type=int, default=min(16, len(os.sched_getaffinity(0))),
                    help="host processes of the CPU baseline, one event each")
    ap.add_argument("--kernels", type=int, default=1,
                    help="also time the fit, backward fit, smoothing and network kernels")
    ap.add_argument("--extended", type=int, default=0,
                    help="also time the seeding pipeline and the material and steering finds")
    ap.add_argument("--field-events", type=int, default=100,
                    help="events of 5,000 tracks for the find in the parameterised field "
                         "with and without the surrogate (0 disables)")
    ap.add_argument("--run-record", default=None,
                    help="append the run record (throughput, roofline fraction, hit-selection "
                         "accuracy, efficiency) as one JSON line to this file")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the find shards by "
              "event with no exchange, so more GPUs would run independent copies of this "
              "workload", file=sys.stderr)
        sys.exit(2)
    forms = [f for f in args.forms.split(",") if f]
    for f in forms:
        if f not in FORMS:
            sys.exit(f"unknown form {f}; known: {', '.join(FORMS)}")

    import numpy as np
    from synth import batched_uneven, generate

    w = batched_uneven(args.events)
    t0 = time.time()
    if args.workload_cache and os.path.exists(args.workload_cache):
        import pickle  # a file this program wrote itself
        with open(args.workload_cache, "rb") as f:
            name, batch = pickle.load(f)
        if name != w.name:
            sys.exit(f"{args.workload_cache} holds {name}, not {w.name}")
        log(f"read {w.name} from {args.workload_cache}")
    else:
        log(f"generating {w.name} with {args.gen_workers} processes")
        batch = generate(w, workers=args.gen_workers)
        if args.workload_cache:
            import pickle
            with open(args.workload_cache, "wb") as f:
                pickle.dump((w.name, batch), f, protocol=pickle.HIGHEST_PROTOCOL)
    log(f"{w.name}: {batch.x.shape[0]} hits, {batch.seed_hits.shape[0]} seeds "
        f"in {time.time() - t0:.1f}s")
    fit_inputs = None
    if args.kernels:  # (in this process: no children under a profiler)
        from synth.fitstress import fit_stress
        fit_inputs = fit_stress(FIT_TRACKS, 26, workers=args.gen_workers)

    import torch
    from paper_1811_04141_amd import mkf
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)  # default priority
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    torch.cuda.synchronize()

    if args.copy_calib:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 x 1 GiB copies")

    train, params = None, None
    if any(f.startswith("surrogate") for f in forms):
        sp = args.surrogate_params
        if sp and os.path.exists(sp):
            params = np.load(sp)  # a plain float32 array this program saved
            train = {"loaded_from": sp}
            log(f"surrogate weights read from {sp}")
        else:
            with torch.cuda.stream(stream):
                c = mkf.Context(w.find, stream=stream.cuda_stream)
                c.load_geometry(w.layers)
                train = c.surrogate_train(**TRAIN)
                params = c.surrogate_get()
                c.close()
            log("surrogate trained", json.dumps(train))
            if sp:
                np.save(sp, params)

    flag_of = {"surrogate": mkf.F_BATCHED | mkf.F_GRAPH | mkf.F_SURROGATE,
               "surrogate_eager": mkf.F_BATCHED | mkf.F_SURROGATE,
               "graph": mkf.F_BATCHED | mkf.F_GRAPH, "batched": mkf.F_BATCHED,
               "plain_all_events": 0}
    results, tracks_ref, ref_name = {}, None, None
    for name in forms:
        if name == "plain_per_event":
            res, tr = time_per_event(mkf, w, batch, stream, args, T)
        else:
            res, tr = time_form(mkf, w, batch, flag_of[name], stream, args, T,
                                params=params if name.startswith("surrogate") else None)
        if tracks_ref is None:
            tracks_ref, ref_name = tr, name
        res["identical_to_" + ref_name] = bool(tr.tobytes() == tracks_ref.tobytes())
        res["same_hits_as_" + ref_name] = float(np.mean(np.all(tr["hit"] == tracks_ref["hit"],
                                                               axis=1)))
        results[name] = res
        log(name, json.dumps(res))
        torch.cuda.empty_cache()

    head = "surrogate" if "surrogate" in results else forms[0]
    R = results[head]
    plain = next((k for k in ("plain_per_event", "plain_all_events") if k in results), None)
    ratios = None
    if plain:
        ratios = {k: {"wall": results[k]["value"] / results[plain]["value"],
                      "device": results[k]["device_value"] / results[plain]["device_value"]}
                  for k in results if k != plain}
        ratios["plain_form"] = plain
    # roofline of the dominant kernel of the headline form, from HIP events on
    # the context stream around its launch (a graph replay cannot bracket the
    # kernel with events: the same kernel's eager form is timed instead)
    eager = {"surrogate": "surrogate_eager", "graph": "batched"}.get(head, head)
    K = results.get(eager, R)
    roof = None
    # the layer-synchronous form's kernel: 6-lane seed groups for budgets up to 6
    plain_kernel = f"k_find_step<false, {6 if w.find.n_cand <= 6 else 8}>"
    if K.get("main_ms", -1) > 0:
        per_launch_steps = K["n_steps"] / max(1, K["main_launches"])
        per_launch_ms = K["main_ms"] / max(1, K["main_launches"])
        if eager.startswith("plain"):
            kname = plain_kernel
            achieved = PLAIN_BYTES_PER_STEP * per_launch_steps / (per_launch_ms * 1e-3) / 1e9
            roof = {"kernel": kname, "bound": "hbm", "achieved": achieved,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s"}
        else:
            t = K["tuning"] or {"waves_per_simd": 0}
            kname = (f"k_find_persistent<{t['waves_per_simd']}, "
                     f"{'true' if eager.startswith('surrogate') else 'false'}, "
                     f"{t.get('lane_group', 6)}>")
            achieved = FLOPS_PER_STEP * per_launch_steps / (per_launch_ms * 1e-3) / 1e12
            roof = {"kernel": kname, "bound": "alu", "achieved": achieved,
                    "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    # the issue limit without packed FP32, which the library is
                    # compiled without: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
                    "peak_unpacked": FP32_VECTOR_PEAK_TFLOPS / 2,
                    "frac_unpacked": achieved / (FP32_VECTOR_PEAK_TFLOPS / 2)}
        roof["frac"] = roof["achieved"] / roof["peak"]
        roof["traffic"] = profiled_traffic(kname, w.name)
        roof["avg_launch_ms"] = per_launch_ms
        roof["timed_form"] = eager
    plain_roof = None
    if "plain_all_events" in results and results["plain_all_events"]["main_ms"] > 0:
        P = results["plain_all_events"]
        gbs = PLAIN_BYTES_PER_STEP * P["n_steps"] / (P["main_ms"] * 1e-3) / 1e9
        per_launch = profiled_traffic(plain_kernel, w.name)
        plain_roof = {"kernel": plain_kernel, "bound": "hbm", "achieved": gbs,
                      "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                      "launches": P["main_launches"], "ms": P["main_ms"],
                      "algorithmic_bytes": PLAIN_BYTES_PER_STEP * P["n_steps"],
                      # all launches of the find, from the profiled per-launch mean
                      "traffic": (per_launch * P["main_launches"]
                                  if per_launch is not None else None)}

    # the found tracks against the generator's truth (hit lists are the same
    # in every form; the plans come from the seeding)
    with torch.cuda.stream(stream):
        cv = mkf.Context(w.find, stream=stream.cuda_stream)
        cv.load_geometry(w.layers)
        cv.load_hits(batch.ev_off, *[T(a) for a in (batch.x, batch.y, batch.z, batch.var_u,
                                                    batch.var_v, batch.layer)])
        cv.seed(T(batch.seed_event), T(batch.seed_hits))
        _, _, s_ok, s_plen, s_plan, _ = cv.get_seed_states(batch.seed_hits.shape[0])
        cv.close()
    val = validation(batch, tracks_ref, s_plen, s_plan, s_ok)
    log("validation", json.dumps(val))
    torch.cuda.empty_cache()

    kernels = (measure_kernels(mkf, w, stream, T, fit_inputs, batch, args.extended, params,
                               args.gen_workers)
               if args.kernels else None)

    field = None
    if args.field_events > 0:
        field = measure_field(mkf, stream, T, args.field_events, args.gen_workers)
        torch.cuda.empty_cache()

    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline(w, batch, args.cpu_seconds, args.cpu_workers)

    line = {
        "metric": METRIC,
        "value": R["value"],
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": R["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "events": w.n_events,
                   "tracks_per_event": "log-uniform 500-20000",
                   "seeds": int(batch.seed_hits.shape[0]), "hits": int(batch.x.shape[0]),
                   "form": head + " (persistent launch, HIP graph, learned surrogate)"
                   if head == "surrogate" else head,
                   "candidates_per_seed": w.find.n_cand},
        "forms": results,
        "vs_plain": ratios,
        "surrogate_training": train,
        "kernels": kernels,
        "field_surrogate": field,
        "validation": val,
        "roofline": roof,
        "plain_roofline": plain_roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    if args.run_record:
        rec = {"time": time.strftime("%Y-%m-%dT%H:%M:%S"), "workload": w.name,
               "value": line["value"], "unit": UNIT,
               "roofline_frac": roof["frac"] if roof else None,
               "plain_hbm_frac": plain_roof["frac"] if plain_roof else None,
               **val}
        with open(args.run_record, "a") as f:
            f.write(json.dumps(rec) + "\n")


if __name__ == "__main__":
    main()
