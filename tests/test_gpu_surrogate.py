"""GPU tests of the learned propagation surrogate through the C ABI: the
matrix-core forward pass and gradients against the FP64 oracle, the
training sampler against the oracle's propagator, training, and the find
with the surrogate against the oracle and against the plain find."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import barrel_endcap, generate
import parity as PT

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NI, NH, NO = O.MLP_NI, O.MLP_NH, O.MLP_NO


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def mkf():
    from paper_1811_04141_amd import mkf as M
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return M


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def glorot(rng, scale=1.0):
    parts = []
    for fo, fi in [(NH, NI), (NH, NH), (NO, NH)]:
        parts.append(rng.normal(size=fo * fi) * scale * np.sqrt(2.0 / (fi + fo)))
        parts.append(rng.normal(size=fo) * 0.1 * scale)
    return np.concatenate(parts).astype(np.float32)


def bf16_weights(p):
    """The parameter vector as the matrix cores see it: weights rounded to
    bfloat16 (round to nearest even, by torch), biases in FP32."""
    q = torch.from_numpy(np.asarray(p, np.float32)).to(torch.bfloat16).float().numpy()
    out = np.asarray(p, np.float64).copy()
    o = 0
    for n, is_w in [(NH * NI, 1), (NH, 0), (NH * NH, 1), (NH, 0), (NO * NH, 1), (NO, 0)]:
        if is_w:
            out[o:o + n] = q[o:o + n]
        o += n
    return out


def samples(mkf, ctx, n, seed):
    x = torch.zeros((n, NI), device="cuda")
    t = torch.zeros((n, NO), device="cuda")
    v = torch.zeros(n, device="cuda")
    ctx.surrogate_samples(n, seed, x, t, v)
    return x, t, v


@pytest.fixture(scope="module")
def geo_ctx(mkf):
    w = barrel_endcap()
    ctx = mkf.Context(w.find, flags=mkf.F_BATCHED | mkf.F_SURROGATE)
    ctx.load_geometry(w.layers)
    yield w, ctx
    ctx.close()


@pytest.fixture(scope="module")
def trained(mkf, geo_ctx):
    w, ctx = geo_ctx
    rep = ctx.surrogate_train(n_samples=1 << 20, epochs=4, batch=512, lr=3e-3, seed=11,
                              loss_w=(1, 0.01, 0.01, 0.01, 0.01, 0.01, 0.01))
    say("training report", rep)
    return rep, ctx.surrogate_get()


@pytest.mark.parametrize("n", [1000, 20000])
def test_infer_matches_oracle(mkf, geo_ctx, n):
    """Both inference layouts (16-sample tiles, the find's own code, for
    calls of up to 16,384 samples; 64-sample tiles above), each on a count
    that is not a multiple of its tile."""
    _, ctx = geo_ctx
    rng = np.random.default_rng(1)
    p = glorot(rng)
    ctx.surrogate_set(p)
    assert np.array_equal(ctx.surrogate_get(), p)
    x, _, _ = samples(mkf, ctx, n, 3)
    y = torch.full((n, NO), np.nan, device="cuda")
    ctx.surrogate_infer(x, y)
    torch.cuda.synchronize()
    xg, yg = x.cpu().numpy(), y.cpu().numpy()
    ref = O.mlp_forward(bf16_weights(p), xg.astype(np.float64), round_bf16=True)
    d = np.abs(yg - ref)
    say("infer max |d|", d.max(), "p99", np.quantile(d, 0.99), "scale", np.abs(ref).max())
    # FP32 against FP64 accumulation; rarely an activation rounds to the
    # neighbouring bfloat16 value (one ulp = 2^-8 relative)
    assert np.quantile(d, 0.99) <= 1e-4
    assert d.max() <= 5e-3


def test_gradient_matches_oracle(mkf, geo_ctx):
    _, ctx = geo_ctx
    rng = np.random.default_rng(2)
    p = glorot(rng)
    ctx.surrogate_set(p)
    n = 512
    x, t, _ = samples(mkf, ctx, n, 4)
    lw = np.array([1.0, 0.5, 0.5, 0.25, 1.0, 1.0, 0.0], np.float32)
    g, L = ctx.surrogate_grad(x, t, lw)
    xr, tr = x.cpu().numpy().astype(np.float64), t.cpu().numpy().astype(np.float64)
    Lr, gr = O.mlp_grad(bf16_weights(p), xr, tr, lw.astype(np.float64), round_bf16=True)
    say("loss gpu", L, "oracle", Lr)
    assert abs(L - Lr) <= 1e-3 * Lr
    # backpropagated errors travel as bfloat16 (8 significant bits) between
    # the matrix-core products: compare block norms
    o = 0
    for name, n_p in [("W1", NH * NI), ("b1", NH), ("W2", NH * NH), ("b2", NH), ("W3", NO * NH),
                      ("b3", NO)]:
        a, b = g[o:o + n_p], gr[o:o + n_p]
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        say(name, "rel err", rel)
        assert rel <= 2e-2, name
        o += n_p


def test_sampler_matches_oracle_propagator(mkf, geo_ctx):
    """Each sample's inputs describe a state up to a rotation about z: put
    it at azimuth 0 and recompute the targets with the oracle's crossing
    and helix transport."""
    w, ctx = geo_ctx
    n = 4096
    x, t, v = samples(mkf, ctx, n, 5)
    xg, tg, vg = (a.cpu().numpy().astype(np.float64) for a in (x, t, v))
    assert vg.mean() >= 0.95
    radii = sorted({l.pos for l in w.layers if l.kind == 0})
    fc = w.find
    mkb = -fc.kappa * fc.bz
    checked = 0
    for i in np.nonzero(vg)[0][:600]:
        R = min(radii, key=lambda r: abs(r - 70.0 * xg[i, 4]))
        assert abs(R - 70.0 * xg[i, 4]) < 1e-4 * R
        r0 = xg[i, 0] * R
        phi = np.arctan2(xg[i, 2], xg[i, 1])
        theta = np.arctan2(1.0, 5.0 * xg[i, 5])
        ipt = xg[i, 7] / 0.3
        om = mkb * ipt
        assert abs(xg[i, 3] - om * R) <= 1e-5 * max(1.0, abs(om * R))
        assert min(abs(r0 - r) for r in radii) < 1e-3 * r0  # starts on a barrel layer
        p = np.array([r0, 0.0, xg[i, 6] * 100.0, ipt, phi, theta])
        l = O.path_to_barrel(p, R, fc.bz, fc.kappa, fc.l_min)
        assert l is not None
        a = r0 * np.cos(phi)
        l_line = -a + np.sqrt(a * a - (r0 * r0 - R * R))
        y0 = 10.0 * (l / l_line - 1.0) / (om * R)
        # FP32 path (and FP32 inputs) to 3e-6 relative, divided by omega R
        assert abs(tg[i, 0] - y0) <= 10 * 3e-6 / abs(om * R) + 1e-4 * abs(y0), (i, tg[i, 0], y0)
        pe = O.transport(p, l, fc.bz, fc.kappa)
        dx, dy = pe[0] - p[0] - l * np.cos(phi), pe[1] - p[1] - l * np.sin(phi)
        along = (dx * np.cos(phi) + dy * np.sin(phi)) * 10.0 / l_line
        across = (dy * np.cos(phi) - dx * np.sin(phi)) * 10.0 / l_line
        assert abs(tg[i, 1] - along) <= 1e-3 and abs(tg[i, 2] - across) <= 1e-3, \
            (i, tg[i], along, across)
        assert abs(tg[i, 4] - 10 * (np.cos(om * l) - 1)) <= 1e-4
        assert abs(tg[i, 5] - 10 * np.sin(om * l)) <= 1e-4
        checked += 1
    assert checked == 600


def test_training_reduces_loss_and_predicts_path(mkf, geo_ctx, trained):
    _, ctx = geo_ctx
    rep, p = trained
    assert rep["n_valid"] >= 0.95 * (1 << 20)
    assert rep["steps"] == 4 * ((1 << 20) // 512)
    assert rep["loss_last"] < 0.01 * rep["loss_first"]
    ctx.surrogate_set(p)
    n = 8192
    x, t, v = samples(mkf, ctx, n, 999)  # held-out seed
    y = torch.zeros((n, NO), device="cuda")
    ctx.surrogate_infer(x, y)
    torch.cuda.synchronize()
    ok = v.cpu().numpy() > 0
    # relative error of the predicted path: |dy0| |omega R| / 10
    err = np.abs(y.cpu().numpy()[ok, 0] - t.cpu().numpy()[ok, 0]) * np.abs(
        x.cpu().numpy()[ok, 3]) / 10.0
    say("held-out relative path error: median", np.median(err), "p90", np.quantile(err, 0.9),
        "frac <= 1e-4", np.mean(err <= 1e-4))
    assert np.median(err) < 1e-4


def run(mkf, w, b, flags, params=None):
    ctx = mkf.Context(w.find, flags=flags)
    ctx.load_geometry(w.layers)
    if params is not None:
        ctx.surrogate_set(params)
    ctx.load_hits(b.ev_off, dev(b.x), dev(b.y), dev(b.z), dev(b.var_u), dev(b.var_v),
                  dev(b.layer))
    ctx.seed(dev(b.seed_event), dev(b.seed_hits))
    ctx.find()
    n = b.seed_hits.shape[0]
    tr = ctx.get_tracks(n)
    st = ctx.stats()
    ctx.close()
    return tr, st


@pytest.mark.parametrize("net", ["trained", "zero", "garbage"])
def test_find_with_surrogate_matches_oracle(mkf, trained, net):
    """Whatever the weights, the found tracks are the plain propagator's:
    a hint is kept only when one Newton step confirms it."""
    w = barrel_endcap()
    b = generate(w, events=[0, 1])
    params = {"trained": trained[1], "zero": np.zeros(O.MLP_NPARAM, np.float32),
              "garbage": glorot(np.random.default_rng(9), scale=8.0)}[net]
    plain, sp = run(mkf, w, b, mkf.F_BATCHED)
    tr, st = run(mkf, w, b, mkf.F_BATCHED | mkf.F_SURROGATE, params)
    kept, rej = st["sur_kept"], st["sur_rejected"]
    say(net, "kept", kept, "rejected", rej, "find ms", st["find_ms"], "plain", sp["find_ms"])
    assert st["n_steps"] > 0 and kept + rej > 0
    assert sp["sur_kept"] == 0 and sp["sur_rejected"] == 0
    if net == "trained":  # 0.68 measured with this training
        assert kept >= 0.5 * (kept + rej)
    # against the oracle on a sample of seeds
    rng = np.random.default_rng(8)
    for e in range(2):
        sel = np.nonzero(b.seed_event == e)[0]
        pick = np.sort(rng.choice(sel, 100, replace=False))
        ref = O.find_event(w.find, w.layers, b.events[e], seeds=b.events[e].seeds[pick - sel[0]])
        out = PT.compare_tracks(tr[pick], ref, mkf.unpack_cov)
        say({k: (v if k != "fail" else len(v)) for k, v in out.items()})
        assert not out["fail"], out["fail"][:5]
        assert out["tie_diverged"] + out["plan_diverged"] <= 0.05 * out["n"] + 1
    # against the plain find on every seed: the same hits, parameters within
    # FP32 rounding of the path length
    same = np.all(tr["hit"] == plain["hit"], axis=1)
    say("identical hit lists", same.mean())
    assert same.mean() >= 0.995
    assert np.array_equal(tr["status"], plain["status"])
    for i in np.nonzero(same)[0]:
        assert PT.par_ok(tr["par"][i], plain["par"][i])[0], (i, tr["par"][i], plain["par"][i])


def test_adam_step_and_schedule_match_oracle(mkf, geo_ctx):
    """One training step at the start, middle and end of a 32-step
    schedule, from a restored optimizer state: the step's gradient (read
    back from the first moment) against the oracle's gradient of the same
    batch (invalid samples weigh zero, the loss is averaged over the
    batch), and the second moment and the parameters against the oracle's
    Adam step with the oracle's cosine step size."""
    _, ctx = geo_ctx
    n, batch, epochs, lr, seed = 8192, 512, 2, 3e-3, 21
    per_epoch = n // batch
    S = per_epoch * epochs
    lw = np.array([1.0, 0.01, 0.01, 0.01, 0.01, 0.01, 0.01], np.float32)
    x, t, v = samples(mkf, ctx, n, seed)
    xg, tg, vg = (a.cpu().numpy().astype(np.float64) for a in (x, t, v))
    rng = np.random.default_rng(22)
    # the library's hyperparameters are FP32 numbers (1 - 0.999f differs
    # from 0.001 by 1.3e-5 relative): the oracle takes them at those values
    b1, b2, eps = (float(np.float32(v)) for v in (0.9, 0.999, 1e-8))
    for s in (0, 13, S - 1):
        p0 = glorot(rng)
        if s == 0:  # a schedule's first step starts from fresh moments
            m0 = np.zeros_like(p0)
            v0 = np.zeros_like(p0)
        else:
            m0 = (rng.normal(size=p0.size) * 1e-4).astype(np.float32)
            v0 = (rng.uniform(0, 1e-6, size=p0.size)).astype(np.float32)
        ctx.surrogate_set_state(p0, m0, v0, s)
        ctx.surrogate_train(n_samples=n, epochs=epochs, batch=batch, lr=lr, seed=seed,
                            loss_w=lw, first_step=s, n_steps=1)
        p1, m1, v1, step = ctx.surrogate_get_state()
        assert step == s + 1
        g = (m1.astype(np.float64) - b1 * m0) / (1 - b1)
        rows = np.arange((s % per_epoch) * batch, (s % per_epoch + 1) * batch)
        ok = rows[vg[rows] != 0]
        _, gr = O.mlp_grad(bf16_weights(p0), xg[ok], tg[ok], lw.astype(np.float64),
                           round_bf16=True)
        gr *= ok.size / batch
        o = 0
        for name, n_p in [("W1", NH * NI), ("b1", NH), ("W2", NH * NH), ("b2", NH),
                          ("W3", NO * NH), ("b3", NO)]:
            rel = np.linalg.norm(g[o:o + n_p] - gr[o:o + n_p]) / np.linalg.norm(gr[o:o + n_p])
            assert rel <= 2e-2, (s, name, rel)
            o += n_p
        lr_s = O.lr_cosine(lr, S, s)
        pe, me, ve = O.adam(p0.astype(np.float64), m0.astype(np.float64),
                            v0.astype(np.float64), g, s + 1, lr_s, b1, b2, eps)
        np.testing.assert_allclose(v1, ve, rtol=1e-5, atol=1e-30)
        step_e = pe - p0
        d = np.abs(p1.astype(np.float64) - pe)
        bound = 1e-4 * np.abs(step_e) + 2.0 * np.spacing(np.abs(p0).astype(np.float32))
        say("adam step", s, "lr", lr_s, "worst", float((d / bound).max()))
        assert np.all(d <= bound), (s, float((d / bound).max()))


def test_training_resumes_bitwise_from_a_checkpoint(mkf, geo_ctx):
    """A 64-step schedule taken in one call, and taken as 40 steps, a
    checkpoint (weights, moments, step) restored into another context, then
    the remaining 24: the same weights and moments bit for bit."""
    w, ctx = geo_ctx
    cfg = dict(n_samples=16384, epochs=2, batch=512, lr=3e-3, seed=31,
               loss_w=(1, 0.01, 0.01, 0.01, 0.01, 0.01, 0.01))
    p0 = glorot(np.random.default_rng(23))
    ctx.surrogate_set(p0)
    rep = ctx.surrogate_train(**cfg)
    assert rep["steps"] == 64
    full = ctx.surrogate_get_state()
    ctx.surrogate_set(p0)
    ctx.surrogate_train(**cfg, n_steps=40)
    ck = ctx.surrogate_get_state()
    assert ck[3] == 40
    ctx2 = mkf.Context(w.find)
    try:
        ctx2.load_geometry(w.layers)
        with pytest.raises(mkf.MkfError):  # its optimizer is at step 0, not 40
            ctx2.surrogate_train(**cfg, first_step=40)
        ctx2.surrogate_set_state(*ck)
        rep = ctx2.surrogate_train(**cfg, first_step=40)
        assert rep["steps"] == 24
        resumed = ctx2.surrogate_get_state()
    finally:
        ctx2.close()
    for a, b in zip(full[:3], resumed[:3]):
        assert np.array_equal(a, b)
    assert full[3] == resumed[3] == 64


def test_checkpoint_blob_round_trips_and_resumes(mkf, geo_ctx):
    """mkf_surrogate_save/_load: the blob of a 40-step checkpoint restored
    into another context resumes the schedule to the uninterrupted run's
    weights and moments bit for bit; a short buffer reports the size with
    MKF_E_CAPACITY, and a blob of the wrong size or header is refused."""
    import ctypes as C
    w, ctx = geo_ctx
    cfg = dict(n_samples=16384, epochs=2, batch=512, lr=3e-3, seed=37,
               loss_w=(1, 0.01, 0.01, 0.01, 0.01, 0.01, 0.01))
    p0 = glorot(np.random.default_rng(29))
    ctx.surrogate_set(p0)
    ctx.surrogate_train(**cfg)
    full = ctx.surrogate_get_state()
    ctx.surrogate_set(p0)
    ctx.surrogate_train(**cfg, n_steps=40)
    blob = ctx.surrogate_save()
    assert len(blob) == 16 + 3 * 4 * mkf.MLP_NPARAM and blob[:4] == b"MKFS"
    n = C.c_size_t(0)
    small = (C.c_ubyte * 100)()
    assert mkf.lib.mkf_surrogate_save(ctx.h, small, 100, C.byref(n)) == mkf.MKF_E_CAPACITY
    assert n.value == len(blob)
    ctx2 = mkf.Context(w.find)
    try:
        ctx2.load_geometry(w.layers)
        for bad in (blob[:-4], b"MKFX" + blob[4:], blob[:4] + b"\x02" + blob[5:]):
            with pytest.raises(mkf.MkfError) as e:
                ctx2.surrogate_load(bad)
            assert e.value.status == mkf.MKF_E_ARG
        ctx2.surrogate_load(blob)
        ck = ctx2.surrogate_get_state()
        assert ck[3] == 40
        ctx2.surrogate_train(**cfg, first_step=40)
        resumed = ctx2.surrogate_get_state()
    finally:
        ctx2.close()
    for a, b in zip(full[:3], resumed[:3]):
        assert np.array_equal(a, b)
    assert full[3] == resumed[3]
