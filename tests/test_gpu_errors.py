"""Failure edges of the C ABI on the GPU: hits with a non-finite value, a
variance that is not positive or a bad layer id are refused at load (from
host and from device memory) and leave the context usable; a track buffer
shorter than the seed count gets the records that fit, the total, and
MKF_E_CAPACITY; out-of-order calls return MKF_E_ORDER."""
import ctypes as C

import numpy as np
import pytest

from synth import generate, small_barrel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mkf():
    from paper_1811_04141_amd import mkf as M
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return M


def arrays(b):
    return [np.ascontiguousarray(a) for a in (b.x, b.y, b.z, b.var_u, b.var_v, b.layer)]


@pytest.mark.parametrize("where", ["host", "device"])
def test_bad_hits_are_refused(mkf, where):
    w = small_barrel()
    b = generate(w)
    ctx = mkf.Context(w.find)
    try:
        ctx.load_geometry(w.layers)
        good = arrays(b)
        put = (lambda a: torch.from_numpy(a).cuda()) if where == "device" else (lambda a: a)
        cases = [(0, 7, np.nan), (1, 11, np.inf), (2, 3, -np.inf), (3, 5, 0.0), (4, 9, -1e-4),
                 (5, 13, len(w.layers)), (5, 2, -1)]
        for field, i, v in cases:
            bad = [a.copy() for a in good]
            bad[field][i] = v
            with pytest.raises(mkf.MkfError) as e:
                ctx.load_hits(b.ev_off, *[put(a) for a in bad])
            assert e.value.status == mkf.MKF_E_ARG, (field, v)
            # nothing was loaded: seeding needs hits
            with pytest.raises(mkf.MkfError) as e:
                ctx.seed(put(np.ascontiguousarray(b.seed_event)),
                         put(np.ascontiguousarray(b.seed_hits)))
            assert e.value.status == mkf.MKF_E_ORDER
        # the context still works with good hits
        ctx.load_hits(b.ev_off, *[put(a) for a in good])
        ctx.seed(put(np.ascontiguousarray(b.seed_event)), put(np.ascontiguousarray(b.seed_hits)))
        ctx.find()
        assert ctx.get_tracks(b.seed_hits.shape[0])["status"].sum() > 0
    finally:
        ctx.close()


def test_short_track_buffer_reports_capacity(mkf):
    w = small_barrel()
    b = generate(w)
    n = b.seed_hits.shape[0]
    ctx = mkf.Context(w.find)
    try:
        ctx.load_geometry(w.layers)
        with pytest.raises(mkf.MkfError) as e:
            ctx.find()  # before seeding
        assert e.value.status == mkf.MKF_E_ORDER
        ctx.load_hits(b.ev_off, *arrays(b))
        ctx.seed(np.ascontiguousarray(b.seed_event), np.ascontiguousarray(b.seed_hits))
        ctx.find()
        full = ctx.get_tracks(n)
        cap = 37
        out = np.zeros(n, mkf.TRACK_DTYPE)
        total = C.c_int64(-1)
        st = mkf.lib.mkf_get_tracks(ctx.h, C.c_void_p(out.ctypes.data), cap, C.byref(total))
        assert st == mkf.MKF_E_CAPACITY and total.value == n
        assert out[:cap].tobytes() == full[:cap].tobytes()
        assert out[cap:].tobytes() == bytes(out[cap:].nbytes)  # nothing written beyond
        assert mkf.lib.mkf_get_tracks(ctx.h, C.c_void_p(out.ctypes.data), -1,
                                      C.byref(total)) == mkf.MKF_E_ARG
    finally:
        ctx.close()


def host_check(tr, b):
    """The checked find's record invariants, evaluated on the host from the
    returned tracks (FP32 where the device uses FP32): one flag per seed."""
    n = tr.shape[0]
    hit = tr["hit"].astype(np.int64)
    plan = tr["plan"].astype(np.int64)
    plen = tr["plan_len"]
    steps = np.arange(hit.shape[1])[None, :]
    inplan = steps < plen[:, None]
    base = b.ev_off[b.seed_event][:, None]
    nev = (b.ev_off[b.seed_event + 1] - b.ev_off[b.seed_event])[:, None]
    found = inplan & (hit >= 0)
    bad_code = inplan & ~((hit >= 0) | (hit == -1) | (hit == -2) | (hit == -3))
    first_none = np.where((inplan & (hit == -3)).any(axis=1),
                          np.argmax(inplan & (hit == -3), axis=1), plen)
    after = inplan & (steps > first_none[:, None]) & (hit != -3)
    out_of_event = found & (hit >= nev)
    lay = np.asarray(b.layer, np.int64)[np.where(found & ~out_of_event, base + hit, 0)]
    wrong_layer = found & ~out_of_event & (lay != plan)
    cov = tr["cov"].astype(np.float32)
    diag = [0, 6, 11, 15, 18, 20]
    d = cov[:, diag]
    tp = (d[:, 0] + d[:, 1]) + d[:, 2]
    bad_var = (~np.isfinite(d).all(axis=1)) | ~(tp > 0) | \
        (d[:, :3] < np.float32(-1e-5) * tp[:, None]).any(axis=1) | ~(d[:, 3:] > 0).all(axis=1)
    ok = tr["status"] == 1
    bad = np.where(ok,
                   bad_code.any(axis=1) | after.any(axis=1) | out_of_event.any(axis=1)
                   | wrong_layer.any(axis=1)
                   | (tr["n_hits"] != 3 + found.sum(axis=1))
                   | (tr["n_miss"] != (inplan & (hit == -1)).sum(axis=1))
                   | ~(tr["chi2"] >= 0) | ~np.isfinite(tr["chi2"])
                   | ~np.isfinite(tr["par"]).all(axis=1) | bad_var,
                   (tr["n_hits"] != 0) | (tr["n_miss"] != 0))
    return bad


@pytest.mark.parametrize("form", ["plain", "batched", "graph", "surrogate", "material", "field"])
def test_checked_find_passes_and_changes_nothing(mkf, form):
    """MKF_F_CHECKED: every result record of a find meets the invariants the
    device check tests (hits of the seed's event on the plan's layers,
    misses and skips, then none; counts that match the list; finite state,
    positive variances), in every form and extension, and the tracks are
    byte for byte those of the unchecked find."""
    from synth import barrel_endcap, barrel_endcap_field, cms_like_material
    w = {"material": cms_like_material, "field": barrel_endcap_field}.get(form, barrel_endcap)()
    b = generate(w, events=[0, 1])
    flags = {"plain": 0, "batched": mkf.F_BATCHED, "graph": mkf.F_BATCHED | mkf.F_GRAPH,
             "surrogate": mkf.F_BATCHED | mkf.F_SURROGATE, "material": mkf.F_BATCHED,
             "field": mkf.F_BATCHED}[form]
    stream = torch.cuda.Stream()
    out = []
    for extra in (0, mkf.F_CHECKED):
        ctx = mkf.Context(w.find, flags=flags | extra, stream=stream.cuda_stream)
        try:
            ctx.load_geometry(w.layers)
            if form == "material":
                ctx.load_material(w.material)
            if form == "field":
                ctx.load_field(w.field)
            if form == "surrogate":
                ctx.surrogate_set((np.random.default_rng(3).normal(size=mkf.MLP_NPARAM) * 0.1)
                                  .astype(np.float32))
            ctx.load_hits(b.ev_off, *arrays(b))
            ctx.seed(np.ascontiguousarray(b.seed_event), np.ascontiguousarray(b.seed_hits))
            for _ in range(2):  # (the graph form: capture, then a replay)
                try:
                    ctx.find()
                except mkf.MkfError as e:  # records stay readable
                    assert e.status == mkf.MKF_E_NUMERIC and extra
            st = ctx.stats()
            out.append(ctx.get_tracks(b.seed_hits.shape[0]))
        finally:
            ctx.close()
    hb = host_check(out[1], b)
    # the device check counts what the host evaluation of the same
    # invariants finds, and the find meets them
    assert st["n_check_failed"] == int(hb.sum()), (form, st["n_check_failed"], int(hb.sum()))
    assert st["n_check_failed"] == 0, (form, np.nonzero(hb)[0][:5])
    assert out[0].tobytes() == out[1].tobytes()
