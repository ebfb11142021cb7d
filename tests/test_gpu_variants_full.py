"""GPU parity of the find's extended forms at the benchmark's size (100
events x 5,000 tracks, one batched launch, the launch shape the benchmark
times): with the silicon-like material map, with five-region steering, and
in the solenoid-like field on events simulated in it.  60 sampled seeds of
two events each against the oracle.  Needs an MI355X."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import (barrel_endcap, barrel_endcap_field, five_regions, generate, generate_event,
                   material_map)
import parity as PT

pytestmark = pytest.mark.gpu

WORKERS = 8  # event generation processes (sized for a 16-CPU host)
MATERIAL = material_map(120.0, 300.0, 24, 30, 0.015, 0.1)

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


def run_and_compare(M, w, b, setup, oracle_kw, events=(7, 63)):
    ctx = M.Context(w.find, flags=M.F_BATCHED)
    ctx.load_geometry(w.layers)
    setup(ctx)
    ctx.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v),
                  dev(b.layer))
    ctx.seed(dev(b.seed_event), dev(b.seed_hits))
    ctx.find()
    n = b.seed_hits.shape[0]
    tr = ctx.get_tracks(n)
    st = ctx.stats()
    ctx.close()
    say(w.name, "seeds", n, "steps", st["n_steps"], "find ms", st["find_ms"])
    rng = np.random.default_rng(97)
    for e in events:
        E = generate_event(w, e)
        sel = np.nonzero(b.seed_event == e)[0]
        pick = np.sort(rng.choice(sel, 60, replace=False))
        seeds = E.seeds[pick - sel[0]]
        assert np.array_equal(seeds, b.seed_hits[pick])
        ref = O.find_event(w.find, w.layers, E, seeds=seeds, **oracle_kw)
        # tracks that meet a layer nearly tangentially (cos < 0.2 against the
        # normal) get the grazing covariance bound: the surface projection
        # divides by the cosine and FP32 cancels terms 1/cos^2 larger
        graze = np.array([PT.conditioning(w, E, list(sh) + [h for h in r["hit"] if h >= 0]) < 0.2
                          for sh, r in zip(seeds, ref)])
        for g, cov_rel in ((False, PT.COV_REL_FOUND), (True, PT.COV_REL_GRAZING)):
            k = np.nonzero(graze == g)[0]
            if k.size == 0:
                continue
            out = PT.compare_tracks(tr[pick[k]], [ref[j] for j in k], M.unpack_cov, cov_rel)
            say("event", e, "grazing" if g else "", {q: (v if q != "fail" else len(v))
                                                    for q, v in out.items()})
            assert not out["fail"], out["fail"][:5]
            assert out["equal"] >= 0.85 * out["n"]


@pytest.fixture(scope="module")
def bench_batch():
    w = barrel_endcap()
    return w, generate(w, workers=WORKERS)


def test_material_map_full_size(mkf, bench_batch):
    w, b = bench_batch
    run_and_compare(mkf, w, b, lambda c: c.load_material(MATERIAL), {"material": MATERIAL})


def test_five_region_steering_full_size(mkf, bench_batch):
    w, b = bench_batch
    st = five_regions()
    run_and_compare(mkf, w, b, lambda c: c.load_steering(st), {"steering": st})


def test_parameterised_field_full_size(mkf):
    w = barrel_endcap_field(100, 5000)
    b = generate(w, workers=WORKERS)
    run_and_compare(mkf, w, b, lambda c: c.load_field(w.field), {"field": w.field})
