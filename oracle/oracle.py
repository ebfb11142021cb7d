"""TEST INFRASTRUCTURE ONLY: ctypes binding of the FP64 CPU oracle
(mkf_oracle.c).  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this module; the GPU library never does.
"""
import ctypes as C
import os
import subprocess
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mkf_oracle.c")
SRC_MLP = os.path.join(HERE, "mkf_mlp.c")
HDR = os.path.join(HERE, "mkf_oracle.h")
LIB = os.path.join(HERE, "libmkf_oracle.so")

MAX_PLAN = 32
OK, NO_CROSSING, OUT_OF_EXTENT = 0, 1, 2
HIT_MISS, HIT_SKIP, HIT_NONE = -1, -2, -3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math)."""
    srcs = (SRC, SRC_MLP, HDR)
    stale = (not os.path.exists(LIB) or
             os.path.getmtime(LIB) < max(os.path.getmtime(f) for f in srcs))
    if force or stale:
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, SRC, SRC_MLP, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Layer(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pos", C.c_double), ("ext_lo", C.c_double),
                ("ext_hi", C.c_double), ("stereo", C.c_double), ("hole_lo", C.c_double),
                ("hole_hi", C.c_double)]


def _layer(l):
    return Layer(int(l.kind), float(l.pos), float(l.ext_lo), float(l.ext_hi),
                 float(getattr(l, "stereo", 0.0)), float(getattr(l, "hole_lo", 0.0)),
                 float(getattr(l, "hole_hi", 0.0)))


class Region(C.Structure):
    _fields_ = [("eta_lo", C.c_double), ("eta_hi", C.c_double), ("n_layers", C.c_int32),
                ("layers", C.c_int32 * MAX_PLAN)]


class Material(C.Structure):
    _fields_ = [("n_r", C.c_int32), ("n_z", C.c_int32), ("r_max", C.c_double),
                ("z_max", C.c_double), ("mass", C.c_double), ("k_max", C.c_double),
                ("x_x0", C.POINTER(C.c_double)), ("xi", C.POINTER(C.c_double))]


class Field(C.Structure):
    _fields_ = [("b0", C.c_double), ("c_r2", C.c_double), ("c_z2", C.c_double),
                ("c_z4", C.c_double), ("h_max", C.c_double)]


class Cfg(C.Structure):
    _fields_ = [("bz", C.c_double), ("kappa", C.c_double), ("chi2_cut", C.c_double),
                ("ms_sigma", C.c_double), ("edge_margin", C.c_double), ("l_min", C.c_double),
                ("n_cand", C.c_int32), ("max_holes", C.c_int32), ("init_var", C.c_double * 6),
                ("regions", C.POINTER(Region)), ("n_regions", C.c_int32),
                ("material", C.POINTER(Material)), ("field", C.POINTER(Field))]


class SeedOut(C.Structure):
    _fields_ = [("ok", C.c_int32), ("par", C.c_double * 6), ("cov", C.c_double * 36),
                ("plan_len", C.c_int32), ("plan", C.c_int32 * MAX_PLAN),
                ("plan_l", C.c_double * MAX_PLAN), ("plan_fragile", C.c_int32),
                ("chi2", C.c_double)]


class Track(C.Structure):
    _fields_ = [("seed_ok", C.c_int32), ("n_hits", C.c_int32), ("n_miss", C.c_int32),
                ("plan_len", C.c_int32), ("plan", C.c_int32 * MAX_PLAN),
                ("hit", C.c_int32 * MAX_PLAN), ("par", C.c_double * 6),
                ("cov", C.c_double * 36), ("chi2", C.c_double),
                ("fragile_step", C.c_int32), ("n_steps", C.c_int64),
                ("plan_fragile", C.c_int32)]


class Path(C.Structure):
    _fields_ = [("bad_step", C.c_int32), ("n_hits", C.c_int32), ("n_miss", C.c_int32),
                ("chi2", C.c_double), ("max_chi2", C.c_double), ("n_near_cut", C.c_int32),
                ("n_edge", C.c_int32), ("par", C.c_double * 6), ("cov", C.c_double * 36)]


class Seeding(C.Structure):
    _fields_ = [("layer", C.c_int32 * 3), ("pt_min", C.c_double), ("d0_max", C.c_double),
                ("z0_max", C.c_double), ("dz_max", C.c_double)]


class Tol(C.Structure):
    _fields_ = [("chi2_rel", C.c_double), ("chi2_abs", C.c_double), ("pos_tol", C.c_double)]


_lib = None
_D = C.POINTER(C.c_double)
_F = C.POINTER(C.c_float)
_I = C.POINTER(C.c_int32)


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        L = _lib
        L.orc_transport.argtypes = [_D, C.c_double, C.c_double, C.c_double, _D]
        L.orc_path_to_barrel.argtypes = [_D, C.c_double, C.c_double, C.c_double, C.c_double, _D]
        L.orc_path_to_disk.argtypes = L.orc_path_to_barrel.argtypes
        L.orc_propagate.argtypes = [_D, _D, C.POINTER(Layer), C.c_double, C.c_double, C.c_double,
                                    C.c_double, C.c_int, _D, _D, _D, _D]
        L.orc_propagate_f.argtypes = L.orc_propagate.argtypes + [C.POINTER(Field)]
        L.orc_field_bz.argtypes = [C.POINTER(Field), C.c_double, C.c_double, C.c_double]
        L.orc_field_bz.restype = C.c_double
        L.orc_add_ms.argtypes = [_D, C.c_double, _D]
        L.orc_bethe_si.argtypes = [C.c_double, C.c_double]
        L.orc_bethe_si.restype = C.c_double
        L.orc_material_effects.argtypes = [C.POINTER(Cfg), C.c_int, _D, _D, C.c_int, _D]
        L.orc_measure.argtypes = [_D, C.c_int, _D, _D, _D]
        L.orc_chi2.argtypes = [_D, _D, C.c_int, _D, C.c_double, C.c_double, C.c_double, _D]
        L.orc_kf_update.argtypes = [_D, _D, C.c_int, _D, _D, _D, C.c_int, _D]
        L.orc_update_hit.argtypes = [_D, _D, C.c_int, _D, C.c_double, C.c_double, C.c_double,
                                     _D]
        L.orc_seed.argtypes = [C.POINTER(Cfg), C.POINTER(Layer), C.c_int32, _D, _D, _I,
                               C.c_double, C.POINTER(SeedOut)]
        L.orc_find_event.argtypes = [C.POINTER(Cfg), C.POINTER(Tol), C.POINTER(Layer), C.c_int32,
                                     C.c_int32, _F, _F, _F, _F, _F, _I, C.c_int32, _I,
                                     C.POINTER(Track)]
        L.orc_find_prefixes.argtypes = [C.POINTER(Cfg), C.POINTER(Tol), C.POINTER(Layer),
                                        C.c_int32, C.c_int32, _F, _F, _F, _F, _F, _I, _I,
                                        C.c_int32, C.c_int32, _I]
        L.orc_find_prefixes.restype = C.c_int32
        L.orc_follow_path.argtypes = [C.POINTER(Cfg), C.POINTER(Tol), C.POINTER(Layer),
                                      C.c_int32, C.c_int32, _F, _F, _F, _F, _F, _I, _I,
                                      C.c_int32, _I, _I, C.POINTER(Path)]
        L.orc_fit_track.argtypes = [C.POINTER(Cfg), _D, _D, C.c_int32, _I, _D, _D, _D, _D, _D,
                                    _D, _D]
        L.orc_flip.argtypes = [_D, _D]
        L.orc_backward_fit.argtypes = [C.POINTER(Cfg), C.POINTER(Layer), C.c_int32, _F, _F, _F,
                                       _F, _F, _I, _I, C.POINTER(Track), _D, _D, _D, _I]
        L.orc_smooth_track.argtypes = [C.POINTER(Cfg), C.POINTER(Layer), C.c_int32, _F, _F, _F,
                                       _F, _F, C.c_int32, _D, _D, C.POINTER(Track), _I, _D, _D]
        L.orc_triplet_params.argtypes = [C.POINTER(Cfg), C.POINTER(Seeding), _D, _D, _D, _D, _D]
        L.orc_triplet_seeds.argtypes = [C.POINTER(Cfg), C.POINTER(Seeding), C.c_int32, _F, _F, _F,
                                        _I, C.c_int32, C.c_double, C.c_int64, _I, _I,
                                        C.POINTER(C.c_int64)]
        L.orc_triplet_seeds.restype = C.c_int64
        L.orc_duplicates.argtypes = [C.c_int32, C.c_int32, _I, _I, _D, _I, C.c_double, C.c_double,
                                     C.c_double, _I, _I]
        L.orc_duplicates.restype = C.c_int32
        L.orc_clean_seeds.argtypes = [C.c_int32, _I, _I, _D, _D, C.c_double, C.c_double,
                                      C.c_double, C.c_double, _I, _I]
        L.orc_clean_seeds.restype = C.c_int32
        L.orc_mlp_forward.argtypes = [_D, C.c_int, _D, C.c_int, _D]
        L.orc_mlp_grad.argtypes = [_D, C.c_int, _D, _D, _D, C.c_int, _D]
        L.orc_mlp_grad.restype = C.c_double
        L.orc_lr_cosine.argtypes = [C.c_double, C.c_int, C.c_int]
        L.orc_lr_cosine.restype = C.c_double
        L.orc_adam.argtypes = [_D, _D, _D, _D, C.c_int, C.c_int, C.c_double, C.c_double,
                               C.c_double, C.c_double]
    return _lib


# ------------------------------------------------------- surrogate MLP

MLP_NI, MLP_NH, MLP_NO = 8, 64, 7
MLP_NPARAM = MLP_NH * MLP_NI + MLP_NH + MLP_NH * MLP_NH + MLP_NH + MLP_NO * MLP_NH + MLP_NO


def mlp_forward(p, x, round_bf16=False):
    p, x = _d(p, MLP_NPARAM), _d(x)
    B = x.size // MLP_NI
    y = np.zeros(B * MLP_NO)
    lib().orc_mlp_forward(_p(p), B, _p(x), int(round_bf16), _p(y))
    return y.reshape(B, MLP_NO)


def mlp_grad(p, x, t, w, round_bf16=False):
    """(loss, gradient) of L = (1/B) sum_s sum_j w_j (y_sj - t_sj)^2."""
    p, x, t, w = _d(p, MLP_NPARAM), _d(x), _d(t), _d(w, MLP_NO)
    B = x.size // MLP_NI
    g = np.zeros(MLP_NPARAM)
    L = lib().orc_mlp_grad(_p(p), B, _p(x), _p(t), _p(w), int(round_bf16), _p(g))
    return L, g


def adam(p, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    p, m, v = (_d(a).copy() for a in (p, m, v))
    g = _d(g)
    lib().orc_adam(_p(p), _p(m), _p(v), _p(g), p.size, t, lr, b1, b2, eps)
    return p, m, v


def lr_cosine(lr, n_steps, s):
    """Step size of step s of an n_steps-step schedule (half cosine from lr
    to lr / 100)."""
    return float(lib().orc_lr_cosine(float(lr), int(n_steps), int(s)))


def _d(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None:
        assert a.size == n, (a.shape, n)
    return a


def _p(a, t=_D):
    return a.ctypes.data_as(t)


def make_layers(layers) -> "C.Array":
    arr = (Layer * len(layers))()
    for i, l in enumerate(layers):
        arr[i] = _layer(l)
    return arr


def make_material(mm):
    """Material record from a map with n_r, n_z, r_max, z_max, mass, k_max
    and the [n_z][n_r] tables x_x0, xi (taken at FP32, as the library
    receives them)."""
    m = Material()
    m.n_r, m.n_z = int(mm.n_r), int(mm.n_z)
    m.r_max, m.z_max = float(np.float32(mm.r_max)), float(np.float32(mm.z_max))
    m.mass, m.k_max = float(np.float32(mm.mass)), float(np.float32(mm.k_max))
    t = np.ascontiguousarray(np.asarray(mm.x_x0, np.float32), np.float64).reshape(-1)
    x = np.ascontiguousarray(np.asarray(mm.xi, np.float32), np.float64).reshape(-1)
    if t.size != m.n_r * m.n_z or x.size != m.n_r * m.n_z:
        raise ValueError("material tables must hold n_z x n_r bins")
    m.x_x0, m.xi = _p(t), _p(x)
    m._keep = (t, x)
    return m


def make_field(fd):
    """Field record from an object with b0, c_r2, c_z2, c_z4, h_max (taken at
    FP32, as the library receives them)."""
    return Field(*[float(np.float32(getattr(fd, k))) for k in ("b0", "c_r2", "c_z2", "c_z4",
                                                                  "h_max")])


def make_cfg(fc, steering=None, material=None, field=None) -> Cfg:
    """steering: a sequence of regions (eta_lo, eta_hi, layers); the bounds
    are taken at FP32, as the library receives them.  material: a material
    map (make_material), or None for the constant scattering angle."""
    c = Cfg()
    c.bz, c.kappa, c.chi2_cut = fc.bz, fc.kappa, fc.chi2_cut
    c.ms_sigma, c.edge_margin, c.l_min = fc.ms_sigma, fc.edge_margin, fc.l_min
    c.n_cand, c.max_holes = fc.n_cand, fc.max_holes
    for i in range(6):
        c.init_var[i] = fc.init_var[i]
    if steering:
        arr = (Region * len(steering))()
        for r, g in zip(arr, steering):
            r.eta_lo, r.eta_hi = float(np.float32(g.eta_lo)), float(np.float32(g.eta_hi))
            if len(g.layers) > MAX_PLAN:
                raise ValueError("region layer list longer than the plan")
            r.n_layers = len(g.layers)
            for k, L in enumerate(g.layers):
                r.layers[k] = int(L)
        c.regions, c.n_regions = arr, len(steering)
        c._keep = arr
    if material is not None:
        m = make_material(material)
        c.material = C.pointer(m)
        c._keep_m = m
    if field is not None:
        f = make_field(field)
        c.field = C.pointer(f)
        c._keep_f = f
    return c


# ------------------------------------------------------------ primitives

def transport(p, l, bz, kappa):
    p = _d(p, 6)
    out = np.zeros(6)
    lib().orc_transport(_p(p), l, bz, kappa, _p(out))
    return out


def path_to_barrel(p, R, bz, kappa, l_min=1e-4):
    p = _d(p, 6)
    l = np.zeros(1)
    st = lib().orc_path_to_barrel(_p(p), R, bz, kappa, l_min, _p(l))
    return float(l[0]) if st == OK else None


def path_to_disk(p, Z, bz, kappa, l_min=1e-4):
    p = _d(p, 6)
    l = np.zeros(1)
    st = lib().orc_path_to_disk(_p(p), Z, bz, kappa, l_min, _p(l))
    return float(l[0]) if st == OK else None


def propagate(p, Cm, layer, bz, kappa, l_min=1e-4, edge_margin=0.0, check_extent=True,
              field=None):
    """Returns (status, p', C', F, l); in the parameterised field if given."""
    p = _d(p, 6)
    Cm = _d(Cm, 36) if Cm is not None else None
    lay = _layer(layer)
    po, Co, Fo, lo = np.zeros(6), np.zeros(36), np.zeros(36), np.zeros(1)
    fld = C.byref(make_field(field)) if field is not None else None
    st = lib().orc_propagate_f(_p(p), _p(Cm) if Cm is not None else None, C.byref(lay), bz, kappa,
                               l_min, edge_margin, int(check_extent), _p(po),
                               _p(Co) if Cm is not None else None, _p(Fo), _p(lo), fld)
    return st, po, Co.reshape(6, 6), Fo.reshape(6, 6), float(lo[0])


def field_bz(field, x, y, z):
    return float(lib().orc_field_bz(C.byref(make_field(field)), float(x), float(y), float(z)))


def add_ms(p, sigma, Cm):
    p = _d(p, 6)
    out = _d(Cm, 36).copy()
    lib().orc_add_ms(_p(p), sigma, _p(out))
    return out.reshape(6, 6)


def bethe_si(bg, mass):
    """Mean ionisation loss in silicon, GeV cm^2 / g."""
    return float(lib().orc_bethe_si(float(bg), float(mass)))


def material_effects(fc, material, kind, p, Cm, direction=1):
    """Effects of one crossed layer's material on (p, Cm).  Returns (p,
    Cm 6x6, M 6x6)."""
    cfg = make_cfg(fc, material=material)
    p = _d(p, 6).copy()
    Cm = _d(Cm, 36).copy()
    M = np.zeros(36)
    lib().orc_material_effects(C.byref(cfg), int(kind), _p(p), _p(Cm), int(direction), _p(M))
    return p, Cm.reshape(6, 6), M.reshape(6, 6)


def measure(p, kind, hit):
    p, hit = _d(p, 6), _d(hit, 3)
    r, H = np.zeros(2), np.zeros(12)
    ok = lib().orc_measure(_p(p), int(kind), _p(hit), _p(r), _p(H))
    return bool(ok), r, H.reshape(2, 6)


def chi2(p, Cm, kind, hit, var_u, var_v, stereo=0.0):
    p, Cm, hit = _d(p, 6), _d(Cm, 36), _d(hit, 3)
    out = np.zeros(1)
    ok = lib().orc_chi2(_p(p), _p(Cm), int(kind), _p(hit), var_u, var_v, stereo, _p(out))
    return float(out[0]) if ok else None


def kf_update(p, Cm, H, r, V, joseph=False):
    p = _d(p, 6).copy()
    Cm = _d(Cm, 36).copy()
    H = _d(H)
    m = H.size // 6
    r, V = _d(r, m), _d(V, m * m)
    c2 = np.zeros(1)
    lib().orc_kf_update(_p(p), _p(Cm), m, _p(H), _p(r), _p(V), int(joseph), _p(c2))
    return p, Cm.reshape(6, 6), float(c2[0])


def update_hit(p, Cm, kind, hit, var_u, var_v, stereo=0.0):
    p = _d(p, 6).copy()
    Cm = _d(Cm, 36).copy()
    hit = _d(hit, 3)
    c2 = np.zeros(1)
    ok = lib().orc_update_hit(_p(p), _p(Cm), int(kind), _p(hit), var_u, var_v, stereo, _p(c2))
    return bool(ok), p, Cm.reshape(6, 6), float(c2[0])


def seed(fc, layers, h, hv, hl, pos_tol=0.0, steering=None, material=None, field=None):
    cfg = make_cfg(fc, steering, material, field)
    lay = make_layers(layers)
    h, hv = _d(h, 9), _d(hv, 6)
    hl = np.ascontiguousarray(hl, np.int32)
    out = SeedOut()
    lib().orc_seed(C.byref(cfg), lay, len(layers), _p(h), _p(hv), _p(hl, _I), pos_tol,
                   C.byref(out))
    n = out.plan_len
    return {"ok": bool(out.ok), "par": np.array(out.par[:]),
            "cov": np.array(out.cov[:]).reshape(6, 6), "plan": np.array(out.plan[:n], np.int32),
            "plan_l": np.array(out.plan_l[:n]), "plan_fragile": bool(out.plan_fragile),
            "chi2": float(out.chi2)}


DEFAULT_TOL = (1e-3, 1e-2, 1e-3)  # chi2 rel, chi2 abs, cm


def find_event(fc, layers, ev, seeds=None, tol=DEFAULT_TOL, steering=None, material=None,
               field=None):
    """Clone-engine finding for the seeds of one event (all seeds if None),
    with region steering and a material map if given.  Returns a list of
    dicts, one per seed."""
    cfg = make_cfg(fc, steering, material, field)
    lay = make_layers(layers)
    t = Tol(*tol)
    seeds = ev.seeds if seeds is None else seeds
    seeds = np.ascontiguousarray(seeds, np.int32).reshape(-1, 3)
    arrs = [np.ascontiguousarray(a, np.float32) for a in (ev.x, ev.y, ev.z, ev.var_u, ev.var_v)]
    layer = np.ascontiguousarray(ev.layer, np.int32)
    out = (Track * max(1, seeds.shape[0]))()
    rc = lib().orc_find_event(C.byref(cfg), C.byref(t), lay, len(layers), int(layer.shape[0]),
                              *[_p(a, _F) for a in arrs], _p(layer, _I), int(seeds.shape[0]),
                              _p(seeds, _I), out)
    if rc != 0:
        raise ValueError("oracle find failed")
    res = []
    # what the parity checks need to question the oracle about one seed again
    ctx = (cfg, t, lay, len(layers), int(layer.shape[0]), arrs, layer)
    for i in range(seeds.shape[0]):
        o = out[i]
        n = o.plan_len
        res.append({"seed_ok": bool(o.seed_ok), "n_hits": o.n_hits, "n_miss": o.n_miss,
                    "plan": np.array(o.plan[:n], np.int32), "hit": np.array(o.hit[:n], np.int32),
                    "par": np.array(o.par[:]), "cov": np.array(o.cov[:]).reshape(6, 6),
                    "chi2": o.chi2, "fragile_step": o.fragile_step, "n_steps": o.n_steps,
                    "plan_fragile": bool(o.plan_fragile),
                    "_orc": (ctx, seeds[i].copy())})
    return res


def find_prefixes(trk, step, cap=4096):
    """Histories (rows of the plan length) of the candidates the oracle's
    find had alive at plan step `step` of the seed of find_event result
    trk (kept at step - 1, then those retired before it; at step >= plan
    length, the final and all retired ones)."""
    (cfg, t, lay, nl, nh, arrs, layer), sh = trk["_orc"]
    hist = np.zeros((cap, MAX_PLAN), np.int32)
    sh = np.ascontiguousarray(sh, np.int32)
    n = lib().orc_find_prefixes(C.byref(cfg), C.byref(t), lay, nl, nh,
                                *[_p(a, _F) for a in arrs], _p(layer, _I), _p(sh, _I),
                                int(step), cap, _p(hist, _I))
    if n < 0 or n > cap:
        raise ValueError("oracle prefixes failed")
    return hist[:n, :len(trk["plan"])].copy()


def follow_path(trk, hist):
    """Follow the history `hist` (one entry per plan step) of the seed of
    find_event result trk with the oracle's filter and check its decisions.
    Returns (status: 0 valid, 1 invalid, -1 seed or plan mismatch, dict)."""
    (cfg, t, lay, nl, nh, arrs, layer), sh = trk["_orc"]
    plan = np.ascontiguousarray(trk["plan"], np.int32)
    h = np.ascontiguousarray(hist, np.int32)
    if h.shape[0] != plan.shape[0]:
        raise ValueError("history and plan lengths differ")
    sh = np.ascontiguousarray(sh, np.int32)
    out = Path()
    st = lib().orc_follow_path(C.byref(cfg), C.byref(t), lay, nl, nh, *[_p(a, _F) for a in arrs],
                               _p(layer, _I), _p(sh, _I), int(plan.shape[0]),
                               _p(plan, _I) if plan.size else None,
                               _p(h, _I) if h.size else None, C.byref(out))
    return int(st), {"bad_step": out.bad_step, "n_hits": out.n_hits, "n_miss": out.n_miss,
                     "chi2": out.chi2, "max_chi2": out.max_chi2,
                     "n_near_cut": out.n_near_cut, "n_edge": out.n_edge,
                     "par": np.array(out.par[:]), "cov": np.array(out.cov[:]).reshape(6, 6)}


def fit_track(fc, p0, C0, kinds, pos, hits, var_u, var_v, material=None, field=None):
    cfg = make_cfg(fc, material=material, field=field)
    p0, C0 = _d(p0, 6), _d(C0, 36)
    kinds = np.ascontiguousarray(kinds, np.int32)
    n = kinds.shape[0]
    pos, hits = _d(pos, n), _d(hits, 3 * n)
    var_u, var_v = _d(var_u, n), _d(var_v, n)
    po, Co, c2 = np.zeros(6), np.zeros(36), np.zeros(1)
    rc = lib().orc_fit_track(C.byref(cfg), _p(p0), _p(C0), n, _p(kinds, _I), _p(pos), _p(hits),
                             _p(var_u), _p(var_v), _p(po), _p(Co), _p(c2))
    return rc, po, Co.reshape(6, 6), float(c2[0])


def flip(p, Cm=None):
    """The same helix traversed the other way (q/pT, phi + pi, pi - theta)."""
    p = _d(p, 6).copy()
    if Cm is None:
        lib().orc_flip(_p(p), None)
        return p
    Cm = _d(Cm, 36).copy()
    lib().orc_flip(_p(p), _p(Cm))
    return p, Cm.reshape(6, 6)


def backward_fit(fc, layers, ev, seed_hits, trk, material=None, field=None):
    """Backward fit of one found track of event ev (a find_event result
    dict, or any dict with seed_ok, plan, hit, par).  Returns (status, par,
    cov 6x6, chi2, n_updates)."""
    cfg = make_cfg(fc, material=material, field=field)
    lay = make_layers(layers)
    t = Track()
    t.seed_ok = int(bool(trk["seed_ok"]))
    plan = np.asarray(trk["plan"], np.int32)
    hit = np.asarray(trk["hit"], np.int32)
    t.plan_len = int(plan.shape[0])
    for i in range(t.plan_len):
        t.plan[i] = int(plan[i])
        t.hit[i] = int(hit[i])
    for i in range(6):
        t.par[i] = float(trk["par"][i])
    arrs = [np.ascontiguousarray(a, np.float32) for a in (ev.x, ev.y, ev.z, ev.var_u, ev.var_v)]
    layer = np.ascontiguousarray(ev.layer, np.int32)
    sh = np.ascontiguousarray(seed_hits, np.int32).reshape(3)
    po, Co, c2, nu = np.zeros(6), np.zeros(36), np.zeros(1), np.zeros(1, np.int32)
    st = lib().orc_backward_fit(C.byref(cfg), lay, len(layers), *[_p(a, _F) for a in arrs],
                                _p(layer, _I), _p(sh, _I), C.byref(t), _p(po), _p(Co), _p(c2),
                                _p(nu, _I))
    return int(st), po, Co.reshape(6, 6), float(c2[0]), int(nu[0])


def _track_struct(trk):
    t = Track()
    t.seed_ok = int(bool(trk["seed_ok"]))
    plan = np.asarray(trk["plan"], np.int32)
    hit = np.asarray(trk["hit"], np.int32)
    t.plan_len = int(plan.shape[0])
    for i in range(t.plan_len):
        t.plan[i] = int(plan[i])
        t.hit[i] = int(hit[i])
    for i in range(6):
        t.par[i] = float(trk["par"][i])
    return t


def smooth_track(fc, layers, ev, seed_layer, seed_par, seed_cov, trk, material=None,
                 field=None):
    """RTS smoothing of one found track of event ev, starting from the seed
    state (seed_par, seed_cov 6x6) on seed_layer.  Returns (n, layers [n],
    par [n][6], cov [n][6][6]); n <= 0 on failure."""
    cfg = make_cfg(fc, material=material, field=field)
    lay = make_layers(layers)
    t = _track_struct(trk)
    arrs = [np.ascontiguousarray(a, np.float32) for a in (ev.x, ev.y, ev.z, ev.var_u, ev.var_v)]
    sp, sc = _d(seed_par, 6), _d(seed_cov, 36)
    ns = MAX_PLAN + 1
    sl = np.zeros(ns, np.int32)
    po, Co = np.zeros(6 * ns), np.zeros(36 * ns)
    n = lib().orc_smooth_track(C.byref(cfg), lay, len(layers), *[_p(a, _F) for a in arrs],
                               int(seed_layer), _p(sp), _p(sc), C.byref(t), _p(sl, _I), _p(po),
                               _p(Co))
    m = max(n, 0)
    return (int(n), sl[:m].copy(), po.reshape(ns, 6)[:m].copy(),
            Co.reshape(ns, 6, 6)[:m].copy())


def make_seeding(sc) -> Seeding:
    s = Seeding()
    for i in range(3):
        s.layer[i] = int(sc.layers[i])
    s.pt_min, s.d0_max, s.z0_max, s.dz_max = sc.pt_min, sc.d0_max, sc.z0_max, sc.dz_max
    return s


def triplet_params(fc, sc, a, b, c):
    """Returns (passes, margin, [pt, d0, dz, z0, psi_ab, psi_ac, psi_0a])."""
    cfg, s = make_cfg(fc), make_seeding(sc)
    v, m = np.zeros(7), np.zeros(1)
    ok = lib().orc_triplet_params(C.byref(cfg), C.byref(s), _p(_d(a, 3)), _p(_d(b, 3)),
                                  _p(_d(c, 3)), _p(v), _p(m))
    return bool(ok), float(m[0]), v


def triplet_seeds(fc, sc, ev, frag_tol=1e-9, a_only=-1):
    """Brute-force triplet seeds of one event (only those starting at hit
    a_only if >= 0): (triplets [n][3] int32, fragile [n] bool, number of
    near-miss triplets)."""
    cfg, s = make_cfg(fc), make_seeding(sc)
    arrs = [np.ascontiguousarray(a, np.float32) for a in (ev.x, ev.y, ev.z)]
    layer = np.ascontiguousarray(ev.layer, np.int32)
    nf = C.c_int64(0)
    cap = 1 << 16
    while True:
        out = np.zeros((cap, 3), np.int32)
        frag = np.zeros(cap, np.int32)
        n = lib().orc_triplet_seeds(C.byref(cfg), C.byref(s), int(layer.shape[0]),
                                    *[_p(a, _F) for a in arrs], _p(layer, _I), int(a_only),
                                    frag_tol, cap,
                                    _p(out, _I), _p(frag, _I), C.byref(nf))
        if n <= cap:
            return out[:n].copy(), frag[:n].astype(bool), int(nf.value)
        cap = int(n)


def track_hit_sets(tracks, seeds):
    """Hit sets (seed hits and found hits) of find_event results."""
    return [list(s) + [int(h) for h in t["hit"] if h >= 0] if t["seed_ok"] else []
            for t, s in zip(tracks, seeds)]


def duplicates(hit_sets, chi2, seeds, frac=0.5, chi2_tol=(1e-3, 1e-2)):
    """Duplicate flags of tracks given their hit sets, chi2 and seed
    triplets: (dup [n] bool, fragile [n] bool)."""
    n = len(hit_sets)
    stride = max([len(h) for h in hit_sets] + [1])
    H = np.full((max(n, 1), stride), -1, np.int32)
    nh = np.zeros(max(n, 1), np.int32)
    for i, h in enumerate(hit_sets):
        H[i, :len(h)] = h
        nh[i] = len(h)
    c2 = _d(np.asarray(chi2, float).reshape(-1) if n else np.zeros(1))
    sd = np.ascontiguousarray(np.asarray(seeds, np.int32).reshape(-1, 3) if n
                              else np.zeros((1, 3), np.int32))
    dup = np.zeros(max(n, 1), np.int32)
    frag = np.zeros(max(n, 1), np.int32)
    lib().orc_duplicates(n, stride, _p(nh, _I), _p(H, _I), _p(c2), _p(sd, _I), frac,
                         chi2_tol[0], chi2_tol[1], _p(dup, _I), _p(frag, _I))
    return dup[:n].astype(bool), frag[:n].astype(bool)


def clean_seeds(trip, ok, par, chi2, tol_ipt, tol_eta, tol_phi, frag_rel=1e-4):
    """Seed cleaning of one event's seeds: (keep [n] bool, fragile [n] bool)."""
    n = len(trip)
    m = max(n, 1)
    T = np.zeros((m, 3), np.int32)
    T[:n] = np.asarray(trip, np.int32).reshape(-1, 3)
    O_ = np.zeros(m, np.int32)
    O_[:n] = np.asarray(ok, np.int32)
    Pm = np.zeros((m, 6))
    Pm[:n] = np.asarray(par, float).reshape(-1, 6)
    c2 = np.zeros(m)
    c2[:n] = np.asarray(chi2, float)
    keep = np.zeros(m, np.int32)
    frag = np.zeros(m, np.int32)
    lib().orc_clean_seeds(n, _p(T, _I), _p(O_, _I), _p(Pm), _p(c2), tol_ipt, tol_eta, tol_phi,
                          frag_rel, _p(keep, _I), _p(frag, _I))
    return keep[:n].astype(bool), frag[:n].astype(bool)
