"""Degenerate and maximum cases with the find's extensions loaded (material
map, parameterised field, region steering): no seeds; an event without hits
and seeds whose region lists hold only their own layers; a one-bin material
map; and the longest region list (32 cylinders, plans of 29 layers) in both
find forms.  Against the oracle.  Needs an MI355X."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import (BARREL, EventRecipe, FieldMap, FindConfig, Layer, MaterialMap, PION_MASS,
                   Region, Workload, generate, generate_event, make_batch, small_barrel)
from synth.workloads import SIGMA_RPHI, SIGMA_Z
import parity as PT

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ONE_BIN = MaterialMap(1, 1, 200.0, 300.0, np.full((1, 1), 0.02, np.float32),
                      np.full((1, 1), 0.2, np.float32), PION_MASS, 10.0)
FIELD = FieldMap(b0=3.8, c_r2=-1e-6, c_z2=-4.9e-6)


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def mkf():
    from paper_1811_04141_amd import mkf as M
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return M


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run(M, w, b, steering, flags=0):
    ctx = M.Context(w.find, flags=flags)
    ctx.load_geometry(w.layers)
    ctx.load_material(ONE_BIN)
    ctx.load_field(FIELD)
    ctx.load_steering(steering)
    ctx.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v),
                  dev(b.layer))
    ctx.seed(dev(b.seed_event), dev(b.seed_hits))
    ctx.find()
    n = b.seed_hits.shape[0]
    tr = ctx.get_tracks(n)
    st = ctx.stats()
    bf = [torch.zeros((max(n, 1), 6), device="cuda"), torch.zeros((max(n, 1), 21), device="cuda"),
          torch.zeros(max(n, 1), device="cuda"),
          torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")]
    ctx.backward_fit(*bf)
    ns = O.MAX_PLAN + 1
    sm = [torch.zeros((max(n, 1), ns, 6), device="cuda"),
          torch.zeros((max(n, 1), ns, 21), device="cuda"),
          torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")]
    ctx.smooth(*sm)
    torch.cuda.synchronize()
    ctx.close()
    return tr, st, [a.cpu().numpy() for a in bf], [a.cpu().numpy() for a in sm]


def test_no_seeds_and_empty_plans(mkf):
    w = small_barrel()
    ev = generate_event(w, 0)
    from synth.events import Event
    empty = Event(*(a[:0] for a in (ev.x, ev.y, ev.z, ev.var_u, ev.var_v, ev.layer, ev.track)),
                  np.zeros((0, 3), np.int32), np.zeros(0, np.int32), ev.truth_state[:0], [])
    # the only region lists the seed layers: every plan is empty
    st = [Region(-1e30, 1e30, (0, 1, 2))]
    b = make_batch([ev, empty])
    tr, stats, bf, sm = run(mkf, w, b, st)
    ref = O.find_event(w.find, w.layers, ev, steering=st, material=ONE_BIN, field=FIELD)
    out = PT.compare_tracks(tr, ref, mkf.unpack_cov)
    say({k: (v if k != "fail" else len(v)) for k, v in out.items()})
    assert not out["fail"] and out["equal"] == out["n"] == 200
    assert np.all(tr["plan_len"] == 0) and stats["n_steps"] == 0
    # the backward fit runs over the seed hits; the smoother has one surface
    for i, r in enumerate(ref):
        s, p, Cm, c2, _ = O.backward_fit(w.find, w.layers, ev, ev.seeds[i], r, material=ONE_BIN,
                                        field=FIELD)
        assert bf[3][i] == s
        if s == 1:
            assert PT.par_ok(bf[0][i], p)[0] and PT.chi2_ok(bf[2][i], c2)
        assert sm[2][i] == (1 if r["seed_ok"] else 0)
    # no seeds at all
    b0 = make_batch([ev])
    b0.seed_event = b0.seed_event[:0]
    b0.seed_hits = b0.seed_hits[:0]
    tr0, st0, _, _ = run(mkf, w, b0, st)
    assert tr0.shape[0] == 0 and st0["n_steps"] == 0


def test_longest_region_list_both_forms(mkf):
    """32 cylinders, one region listing all of them: plans of 29 layers.
    With the extensions loaded the two forms are bitwise equal too (the
    material and field arithmetic contracts within expressions only, so
    every kernel that inlines it rounds alike) and match the oracle."""
    radii = np.linspace(3.0, 100.0, 32)
    layers = [Layer(BARREL, float(r), -200.0, 200.0, SIGMA_RPHI ** 2, SIGMA_Z ** 2) for r in radii]
    w = Workload(name="barrel32_1x400", layers=tuple(layers),
                 recipe=EventRecipe(pt_lo=1.0, pt_hi=10.0, eta_max=1.0, ms_sigma=0.001,
                                    hit_ineff=0.02, noise_frac=0.3),
                 find=FindConfig(), n_events=1, n_tracks=(400, 400), master_seed=0x5EED0007)
    b = generate(w)
    st = [Region(-1e30, 1e30, tuple(range(32)))]
    a, sa, _, _ = run(mkf, w, b, st, flags=0)
    c, sc, _, _ = run(mkf, w, b, st, flags=mkf.F_BATCHED)
    assert a["plan_len"].max() == 29
    assert sa["n_steps"] == sc["n_steps"] and a.tobytes() == c.tobytes()
    ev = b.events[0]
    rng = np.random.default_rng(5)
    pick = np.sort(rng.choice(len(ev.seeds), 100, replace=False))
    ref = O.find_event(w.find, w.layers, ev, seeds=ev.seeds[pick], steering=st,
                       material=ONE_BIN, field=FIELD)
    out = PT.compare_tracks(a[pick], ref, mkf.unpack_cov)
    say({k: (v if k != "fail" else len(v)) for k, v in out.items()})
    assert not out["fail"] and out["equal"] >= 0.9 * out["n"]


def test_largest_material_map_and_fine_field_steps(mkf):
    """A 2048 x 2047-bin material map with a different thickness in every bin
    (above what the persistent find stages in LDS, so it reads the table
    from HBM) and field steps of 0.05 cm, on the small barrel event, in both
    find forms: equal to each other and to the oracle.  A crossing on a bin
    edge may take either bin (FP32 against FP64), so the map's radial edges
    are kept off the layer radii (at least 5e-4 cm away): 2047 bins over
    200 cm rather than 2048, which would put an edge at R = 25 cm."""
    from dataclasses import replace
    w = small_barrel()
    ev = generate_event(w, 0)
    nr, nz = 2047, 2048
    rng = np.random.default_rng(11)
    big = MaterialMap(nr, nz, 200.0, 300.0,
                      rng.uniform(0.005, 0.03, (nz, nr)).astype(np.float32),
                      rng.uniform(0.05, 0.3, (nz, nr)).astype(np.float32), PION_MASS, 10.0)
    edges = np.array([L.pos for L in w.layers]) * nr / 200.0
    assert np.all(np.abs(edges - np.round(edges)) * 200.0 / nr > 5e-4)
    fine = replace(FIELD, h_max=0.05)
    b = make_batch([ev])
    out = []
    for flags in (0, mkf.F_BATCHED):
        ctx = mkf.Context(w.find, flags=flags)
        ctx.load_geometry(w.layers)
        ctx.load_material(big)
        ctx.load_field(fine)
        ctx.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v),
                      dev(b.layer))
        ctx.seed(dev(b.seed_event), dev(b.seed_hits))
        ctx.find()
        out.append(ctx.get_tracks(b.seed_hits.shape[0]))
        ctx.close()
    assert out[0].tobytes() == out[1].tobytes()
    ref = O.find_event(w.find, w.layers, ev, material=big, field=fine)
    res = PT.compare_tracks(out[1], ref, mkf.unpack_cov)
    say({k: (v if k != "fail" else len(v)) for k, v in res.items()})
    assert not res["fail"] and res["equal"] >= 0.95 * res["n"]
