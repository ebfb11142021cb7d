"""Throughput of the Kalman-filter track finding hot path on one MI355X.

A step is one pass of the find (propagate, hit search, chi2, per-seed
selection, Kalman update over every plan layer of every seed) over the whole
workload: 100 synthetic barrel+endcap events of 5,000 tracks (scattering,
2% inefficiency, 30% noise hits).  Hits are indexed and seeds fitted before
the timed region (the paper times core finding without this
pre-processing, Section 4.1); inputs are resident in HBM.

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
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
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
BF16_MFMA_PEAK_TFLOPS = 2500.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def profiled_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter record
    (FETCH_SIZE and WRITE_SIZE, scaled by a 1 GiB copy), or None if the
    kernel sources changed since the counters were taken."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")):
        rec = json.load(open(path))
        if not rec["kernel"].startswith(kernel):
            continue
        h = hashlib.sha256()
        for f in rec["sources"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() == rec["source_sha256"]:
            return rec["hbm_bytes_per_launch"]
    return None


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
    """The FP64 oracle as it stands, one event per host thread (the paper's
    events-in-flight pattern), each on its own process; throughput is the
    summed steps over the longest worker's time."""
    n = max(1, min(workers, len(batch.events)))
    jobs = [(w, batch.events[e], seconds) for e in range(n)]
    if n == 1:
        out = [_oracle_share(jobs[0])]
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
    return {"value": steps / t, "unit": UNIT, "cores": n, "kind": "oracle",
            "sample": f"first seeds of events 0-{n - 1}, one event per process "
                      f"({seeds} seeds, {steps} candidate-layer steps, {t:.1f} s; FP64, "
                      f"brute-force hit scan)"}


def measure_kernels(mkf, w, stream, T, f, batch, hits, seeds):
    """Throughput of the other hot-path kernels, each from HIP events on the
    context stream around one launch after a warm-up: the search-free fit
    (131,072 tracks x 26 layers), the backward fit and the smoothing of the
    benchmark workload's found tracks, triplet seeding with cleaning, find and
    duplicate removal on it, the find with a material map and with region
    steering, the find in a parameterised field (events simulated in it),
    and the surrogate network's inference and gradient (2^20 samples from
    its training sampler)."""
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

    out = {}
    with torch.cuda.stream(stream):
        ctx = mkf.Context(w.find, stream=stream.cuda_stream)
        ctx.load_geometry(w.layers)
        k, n = f.x.shape
        ins = [T(a) for a in (f.kind, f.pos, f.x, f.y, f.z, f.var_u, f.var_v, f.length,
                              f.init_par, f.init_cov)]
        outs = [torch.zeros((n, 6), device=ins[0].device), torch.zeros((n, 21), device=ins[0].device),
                torch.zeros(n, device=ins[0].device),
                torch.zeros(n, dtype=torch.int32, device=ins[0].device)]
        ms = timed(lambda: ctx.fit(*ins, *outs))
        out["k_fit"] = dict(alu(FIT_FLOPS_PER_UPDATE * n * k, ms, FP32_VECTOR_PEAK_TFLOPS, n * k,
                                "track-layer updates/s"), bound="alu",
                            workload=f"{n} tracks x {k} layers")
        # backward fit of the tracks found in the benchmark workload,
        # counted by its updates (one per hit, the seed hits included; the
        # propagations through layers without a hit are not counted)
        ctx2 = mkf.Context(w.find, flags=mkf.F_BATCHED, stream=stream.cuda_stream)
        ctx2.load_geometry(w.layers)
        ctx2.load_hits(batch.ev_off, *hits)
        ctx2.seed(*seeds)
        ctx2.find()
        ns = batch.seed_hits.shape[0]
        tr = ctx2.get_tracks(ns)
        dev = ins[0].device
        bouts = [torch.zeros((ns, 6), device=dev), torch.zeros((ns, 21), device=dev),
                 torch.zeros(ns, device=dev), torch.zeros(ns, dtype=torch.int32, device=dev)]
        ms = timed(lambda: ctx2.backward_fit(*bouts))
        ok = bouts[3].cpu().numpy() == 1
        upd = int(tr["n_hits"][ok].sum())
        out["k_backfit"] = dict(alu(FIT_FLOPS_PER_UPDATE * upd, ms, FP32_VECTOR_PEAK_TFLOPS, upd,
                                    "track-hit updates/s"), bound="alu",
                                workload=f"{int(ok.sum())} found tracks, {upd} hits")
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
        # combinatorial triplet seeding, seed cleaning, the find from all the
        # triplet seeds and duplicate removal on the same workload (each call
        # between HIP events on the context stream; the seeding and removal
        # calls wait on the host for their counts inside that span)
        from synth import CleaningConfig, SeedingConfig
        ctx3 = mkf.Context(w.find, flags=mkf.F_BATCHED, stream=stream.cuda_stream)
        ctx3.load_geometry(w.layers)
        ctx3.load_hits(batch.ev_off, *hits)
        cap = 8 << 20
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
        # the batched find with a silicon-like material map (1.5% of a
        # radiation length and 0.1 g/cm^2 per layer, 1.5x beyond |z| = 50 cm)
        # and with five-region steering, from the same seeds (each autotuned;
        # mkf_get_stats timing)
        from synth import five_regions, material_map
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
                          "unit": "candidate-layer updates/s", "workload": w.name,
                          "tuning": tun4}
        # the batched find in the solenoid-like parameterised field (Runge-Kutta
        # crossings) on events of the benchmark's sizes simulated in that field
        # (generated here, in this process: ~1.6 s per event), against the
        # uniform-field find on the same events
        from synth import barrel_endcap_field, generate_event, make_batch
        wf = barrel_endcap_field(w.n_events, w.n_tracks[0])
        evs = []
        for e in range(wf.n_events):
            evs.append(generate_event(wf, e))
            if e % 10 == 9:
                log(f"field events generated: {e + 1}/{wf.n_events}")
        bf = make_batch(evs)
        del evs
        fh = [T(a) for a in (bf.x, bf.y, bf.z, bf.var_u, bf.var_v, bf.layer)]
        fs = (T(bf.seed_event), T(bf.seed_hits))
        for label, fld in (("find_parameterised_field", wf.field),
                           ("find_uniform_field_same_events", None)):
            c5 = mkf.Context(wf.find, flags=mkf.F_BATCHED, stream=stream.cuda_stream)
            c5.load_geometry(wf.layers)
            c5.load_field(fld)
            c5.load_hits(bf.ev_off, *fh)
            c5.seed(*fs)
            tun5 = c5.autotune(repeats=2)
            c5.find()
            c5.find()
            st = c5.stats()
            n = int(bf.seed_hits.shape[0])
            tr = c5.get_tracks(n)
            c5.close()
            out[label] = {"find_ms": st["find_ms"], "n_steps": st["n_steps"],
                          "throughput": st["n_steps"] / (st["find_ms"] * 1e-3),
                          "unit": "candidate-layer updates/s", "workload": wf.name,
                          "mean_hits_per_track": float(tr["n_hits"].mean()), "tuning": tun5}
        del fh, fs, bf
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
        ctx.close()
    log("kernels", json.dumps(out))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=100)
    ap.add_argument("--tracks", type=int, default=5000)
    ap.add_argument("--forms", default="plain,batched,graph,surrogate")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="budget of the oracle CPU baseline (0 disables)")
    ap.add_argument("--cpu-workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="host processes of the CPU baseline, one event each")
    ap.add_argument("--kernels", type=int, default=1,
                    help="also time the fit and the surrogate network kernels (0 disables)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the find shards by "
              "event with no exchange, so more GPUs would run independent copies of this "
              "workload", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    from synth import barrel_endcap, generate

    w = barrel_endcap(args.events, args.tracks)
    t0 = time.time()
    batch = generate(w)
    log(f"generated {w.name}: {batch.x.shape[0]} hits, {batch.seed_hits.shape[0]} seeds "
        f"in {time.time() - t0:.1f}s")
    fit_inputs = None
    if args.kernels:  # (in this process: no children under a profiler)
        from synth.fitstress import fit_stress
        fit_inputs = fit_stress(131072, 26)

    import torch
    from paper_1811_04141_amd import mkf
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)  # default priority
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    hits = [T(a) for a in (batch.x, batch.y, batch.z, batch.var_u, batch.var_v, batch.layer)]
    seeds = (T(batch.seed_event), T(batch.seed_hits))
    torch.cuda.synchronize()

    if args.copy_calib:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 1 GiB copies")

    forms = {"plain": 0, "batched": mkf.F_BATCHED, "graph": mkf.F_BATCHED | mkf.F_GRAPH,
             "surrogate": mkf.F_BATCHED | mkf.F_GRAPH | mkf.F_SURROGATE}
    results = {}
    tracks_ref = None
    for name in args.forms.split(","):
        flags = forms[name]
        with torch.cuda.stream(stream):
            ctx = mkf.Context(w.find, flags=flags, stream=stream.cuda_stream)
            ctx.load_geometry(w.layers)
            train = None
            if flags & mkf.F_SURROGATE:  # trained on the GPU before the timed region
                train = ctx.surrogate_train(n_samples=1 << 20, epochs=4, batch=512, lr=3e-3,
                                            seed=11, loss_w=(1, .01, .01, .01, .01, .01, .01))
            ctx.load_hits(batch.ev_off, *hits)
            ctx.seed(*seeds)
            tuning = ctx.autotune(repeats=2) if flags & mkf.F_BATCHED else None
            for _ in range(args.warmup):
                ctx.find()
            torch.cuda.synchronize()
            main_ms = []
            find_ms = []
            t_start = time.perf_counter()
            for _ in range(args.steps):
                ctx.find()
                st = ctx.stats()
                main_ms.append(st["main_ms"])
                find_ms.append(st["find_ms"])
            torch.cuda.synchronize()
            t_end = time.perf_counter()
            n_seeds = batch.seed_hits.shape[0]
            tr = ctx.get_tracks(n_seeds)
            if tracks_ref is None:
                tracks_ref = tr
            same = tr.tobytes() == tracks_ref.tobytes()
            st = ctx.stats()
            ctx.close()
        wall = (t_end - t_start) / args.steps
        results[name] = {
            "ms_per_step": wall * 1e3,
            "find_ms": float(np.mean(find_ms)),
            "main_ms": float(np.mean(main_ms)),
            "main_launches": st["main_launches"],
            "n_steps": st["n_steps"],
            "value": st["n_steps"] / wall,
            "identical_to_first_form": bool(same),
            "same_hits_as_first_form": float(np.mean(np.all(tr["hit"] == tracks_ref["hit"],
                                                            axis=1))),
            "tuning": tuning,
        }
        if train is not None:
            results[name]["surrogate"] = {
                "kept": st["sur_kept"], "rejected": st["sur_rejected"],
                "kept_frac": st["sur_kept"] / max(1, st["sur_kept"] + st["sur_rejected"]),
                "train": train}
        log(name, json.dumps(results[name]))

    best = max(results, key=lambda k: results[k]["value"])
    speedup = None
    if "surrogate" in results and "plain" in results:
        speedup = {k: results["surrogate"]["value"] / results[k]["value"]
                   for k in ("plain", "batched", "graph") if k in results}
    R = results[best]
    # roofline of the dominant kernel, from HIP events on the context stream
    # (a graph replay cannot bracket the kernel with events: take the same
    # kernel's eager form, else the whole find of the best form)
    timed = [k for k in (best, "batched", "plain") if k in results and results[k]["main_ms"] > 0]
    kernel_form = timed[0] if timed else best
    K = results[kernel_form]
    kernel_ms = K["main_ms"] if K["main_ms"] > 0 else K["find_ms"]
    per_launch_steps = K["n_steps"] / max(1, K["main_launches"])
    per_launch_ms = kernel_ms / max(1, K["main_launches"])
    if kernel_form == "plain":
        achieved = PLAIN_BYTES_PER_STEP * per_launch_steps / (per_launch_ms * 1e-3) / 1e9
        roof = {"kernel": "k_find_step", "bound": "hbm", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        achieved = FLOPS_PER_STEP * per_launch_steps / (per_launch_ms * 1e-3) / 1e12
        roof = {"kernel": "k_find_persistent", "bound": "alu", "achieved": achieved,
                "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = profiled_traffic(roof["kernel"])
    roof["avg_launch_ms"] = per_launch_ms

    kernels = (measure_kernels(mkf, w, stream, T, fit_inputs, batch, hits, seeds)
               if args.kernels else None)

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
        "config": {"workload": w.name, "events": args.events, "tracks_per_event": args.tracks,
                   "seeds": int(batch.seed_hits.shape[0]), "hits": int(batch.x.shape[0]),
                   "form": best, "candidates_per_seed": w.find.n_cand},
        "forms": results,
        "surrogate_speedup": speedup,
        "kernels": kernels,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
