"""ctypes binding of libmkf.so (C ABI in include/mkf.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Device arrays are torch tensors on the GPU (PyTorch provides device
memory and streams); host arrays are numpy arrays.  There is no CPU fallback:
if the library is missing this module raises on import.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmkf.so")

MKF_OK, MKF_E_ARG, MKF_E_ORDER, MKF_E_CAPACITY, MKF_E_HIP, MKF_E_GEOMETRY, MKF_E_NUMERIC = (
    0, -1, -2, -3, -4, -5, -6)
MEM_HOST, MEM_DEVICE = 0, 1
F_BATCHED, F_GRAPH, F_SURROGATE, F_CHECKED = 1, 2, 4, 8
MLP_NPARAM = 5191  # W1[64][8], b1[64], W2[64][64], b2[64], W3[7][64], b3[7]
NOALLOC_MAX_SAMPLES = 16384  # MKF_NOALLOC_MAX_SAMPLES
MAX_LAYERS = MAX_PLAN = 32
MAX_CAND = 8
MAX_REGIONS = 8
HIT_MISS, HIT_SKIP, HIT_NONE = -1, -2, -3

EXPORTS = ("mkf_create", "mkf_destroy", "mkf_last_error", "mkf_load_geometry",
           "mkf_load_steering", "mkf_load_material", "mkf_load_field", "mkf_load_hits",
           "mkf_seed", "mkf_get_seed_states", "mkf_find", "mkf_get_tracks", "mkf_propagate",
           "mkf_fit", "mkf_backward_fit", "mkf_smooth", "mkf_make_seeds", "mkf_clean_seeds",
           "mkf_find_duplicates",
           "mkf_get_stats",
           "mkf_set_tuning",
           "mkf_get_tuning", "mkf_autotune", "mkf_surrogate_train", "mkf_surrogate_get", "mkf_surrogate_set",
           "mkf_surrogate_get_state", "mkf_surrogate_set_state", "mkf_surrogate_save", "mkf_surrogate_load", "mkf_surrogate_grad",
           "mkf_surrogate_grad_noalloc",
           "mkf_surrogate_infer", "mkf_surrogate_samples")


class MkfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mkf status {status}: {msg}")
        self.status = status


class Layer(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pos", C.c_float), ("ext_lo", C.c_float),
                ("ext_hi", C.c_float), ("var_u_max", C.c_float), ("var_v_max", C.c_float),
                ("n_phi_bins", C.c_int32), ("n_q_bins", C.c_int32), ("stereo", C.c_float),
                ("hole_lo", C.c_float), ("hole_hi", C.c_float)]


class Config(C.Structure):
    _fields_ = [("bz", C.c_float), ("kappa", C.c_float), ("chi2_cut", C.c_float),
                ("ms_sigma", C.c_float), ("edge_margin", C.c_float), ("l_min", C.c_float),
                ("n_cand", C.c_int32), ("max_holes", C.c_int32), ("init_var", C.c_float * 6),
                ("flags", C.c_uint32)]


class Track(C.Structure):
    _fields_ = [("seed_id", C.c_int32), ("status", C.c_int32), ("n_hits", C.c_int32),
                ("n_miss", C.c_int32), ("plan_len", C.c_int32), ("chi2", C.c_float),
                ("par", C.c_float * 6), ("cov", C.c_float * 21), ("plan", C.c_int8 * MAX_PLAN),
                ("hit", C.c_int32 * MAX_PLAN)]


TRACK_DTYPE = np.dtype([("seed_id", "<i4"), ("status", "<i4"), ("n_hits", "<i4"),
                        ("n_miss", "<i4"), ("plan_len", "<i4"), ("chi2", "<f4"),
                        ("par", "<f4", 6), ("cov", "<f4", 21), ("plan", "i1", MAX_PLAN),
                        ("hit", "<i4", MAX_PLAN)], align=True)
assert TRACK_DTYPE.itemsize == C.sizeof(Track)


class Seeding(C.Structure):
    _fields_ = [("layers", C.c_int32 * 3), ("pt_min", C.c_float), ("d0_max", C.c_float),
                ("z0_max", C.c_float), ("dz_max", C.c_float)]


def make_seeding(sc):
    s = Seeding()
    for i in range(3):
        s.layers[i] = int(sc.layers[i])
    s.pt_min, s.d0_max, s.z0_max, s.dz_max = sc.pt_min, sc.d0_max, sc.z0_max, sc.dz_max
    return s


class Region(C.Structure):
    _fields_ = [("eta_lo", C.c_float), ("eta_hi", C.c_float), ("n_layers", C.c_int32),
                ("layers", C.c_int32 * MAX_PLAN)]


def make_regions(regions):
    """Region records from objects with eta_lo, eta_hi and layers."""
    arr = (Region * max(1, len(regions)))()
    for r, g in zip(arr, regions):
        if len(g.layers) > MAX_PLAN:
            raise ValueError("a region lists more than %d layers" % MAX_PLAN)
        r.eta_lo, r.eta_hi, r.n_layers = g.eta_lo, g.eta_hi, len(g.layers)
        for k, L in enumerate(g.layers):
            r.layers[k] = int(L)
    return arr


class MaterialInfo(C.Structure):
    _fields_ = [("n_r", C.c_int32), ("n_z", C.c_int32), ("r_max", C.c_float),
                ("z_max", C.c_float), ("mass", C.c_float), ("k_max", C.c_float)]


class Field(C.Structure):
    _fields_ = [("b0", C.c_float), ("c_r2", C.c_float), ("c_z2", C.c_float),
                ("c_z4", C.c_float), ("h_max", C.c_float)]


class Cleaning(C.Structure):
    _fields_ = [("tol_ipt", C.c_float), ("tol_eta", C.c_float), ("tol_phi", C.c_float)]


class Stats(C.Structure):
    _fields_ = [("n_seeds", C.c_int64), ("n_seeds_ok", C.c_int64), ("n_steps", C.c_int64),
                ("max_plan_len", C.c_int32), ("n_launches", C.c_int32), ("find_ms", C.c_float),
                ("index_ms", C.c_float), ("seed_ms", C.c_float), ("main_ms", C.c_float),
                ("main_launches", C.c_int32), ("sur_kept", C.c_int64),
                ("sur_rejected", C.c_int64), ("n_near_cut", C.c_int64),
                ("n_rk_steps", C.c_int64), ("n_newton", C.c_int64),
                ("n_check_failed", C.c_int64)]


class TrainCfg(C.Structure):
    _fields_ = [("n_samples", C.c_int64), ("epochs", C.c_int32), ("batch", C.c_int32),
                ("lr", C.c_float), ("seed", C.c_uint64), ("loss_w", C.c_float * 7),
                ("first_step", C.c_int32), ("n_steps", C.c_int32)]


class TrainReport(C.Structure):
    _fields_ = [("steps", C.c_int32), ("loss_first", C.c_float), ("loss_last", C.c_float),
                ("datagen_ms", C.c_float), ("train_ms", C.c_float), ("n_valid", C.c_int64)]


class Tuning(C.Structure):
    _fields_ = [("waves_per_simd", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("lane_group", C.c_int32), ("phi_bin_shift", C.c_int32),
                ("q_bin_shift", C.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    P, I64, I32, U32 = C.c_void_p, C.c_int64, C.c_int32, C.c_uint32
    sig = {
        "mkf_create": ([C.POINTER(Config), P, C.POINTER(P)], I32),
        "mkf_destroy": ([P], None),
        "mkf_last_error": ([P], C.c_char_p),
        "mkf_load_geometry": ([P, C.POINTER(Layer), I32], I32),
        "mkf_load_steering": ([P, C.POINTER(Region), I32], I32),
        "mkf_load_material": ([P, C.POINTER(MaterialInfo), P, P], I32),
        "mkf_load_field": ([P, C.POINTER(Field)], I32),
        "mkf_load_hits": ([P, I32, P, P, P, P, P, P, P, I32], I32),
        "mkf_seed": ([P, I64, P, P, I32], I32),
        "mkf_get_seed_states": ([P, P, P, P, P, P, P], I32),
        "mkf_find": ([P], I32),
        "mkf_get_tracks": ([P, P, I64, C.POINTER(I64)], I32),
        "mkf_propagate": ([P, I64, P, P, P, P, P, P, P], I32),
        "mkf_fit": ([P, I64, I32, P, P, P, P, P, P, P, P, P, P, P, P, P, P], I32),
        "mkf_backward_fit": ([P, P, P, P, P], I32),
        "mkf_smooth": ([P, P, P, P], I32),
        "mkf_make_seeds": ([P, C.POINTER(Seeding), I64, P, P, C.POINTER(I64)], I32),
        "mkf_find_duplicates": ([P, C.c_float, P, C.POINTER(I64)], I32),
        "mkf_clean_seeds": ([P, C.POINTER(Cleaning), P, C.POINTER(I64)], I32),
        "mkf_get_stats": ([P, C.POINTER(Stats)], I32),
        "mkf_set_tuning": ([P, C.POINTER(Tuning)], I32),
        "mkf_get_tuning": ([P, C.POINTER(Tuning)], I32),
        "mkf_autotune": ([P, I32, C.c_char_p, C.POINTER(Tuning)], I32),
        "mkf_surrogate_train": ([P, C.POINTER(TrainCfg), C.POINTER(TrainReport)], I32),
        "mkf_surrogate_get": ([P, P], I32),
        "mkf_surrogate_set": ([P, P], I32),
        "mkf_surrogate_get_state": ([P, P, P, P, C.POINTER(I32)], I32),
        "mkf_surrogate_set_state": ([P, P, P, P, I32], I32),
        "mkf_surrogate_save": ([P, P, C.c_size_t, C.POINTER(C.c_size_t)], I32),
        "mkf_surrogate_load": ([P, P, C.c_size_t], I32),
        "mkf_surrogate_grad": ([P, I32, P, P, P, P, P], I32),
        "mkf_surrogate_grad_noalloc": ([P, I32, P, P, P, P, P], I32),
        "mkf_surrogate_infer": ([P, I64, P, P], I32),
        "mkf_surrogate_samples": ([P, I64, C.c_uint64, P, P, P], I32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()


def _ptr(a):
    """Address of a torch tensor (device) or numpy array (host)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        assert a.is_contiguous()
        return C.c_void_p(a.data_ptr())
    assert a.flags["C_CONTIGUOUS"]
    return C.c_void_p(a.ctypes.data)


def _is_device(a):
    return hasattr(a, "is_cuda") and a.is_cuda


def make_config(fc, flags=0):
    c = Config()
    c.bz, c.kappa, c.chi2_cut = fc.bz, fc.kappa, fc.chi2_cut
    c.ms_sigma, c.edge_margin, c.l_min = fc.ms_sigma, fc.edge_margin, fc.l_min
    c.n_cand, c.max_holes = fc.n_cand, fc.max_holes
    for i in range(6):
        c.init_var[i] = fc.init_var[i]
    c.flags = flags
    return c


def make_layers(layers):
    arr = (Layer * len(layers))()
    for i, l in enumerate(layers):
        arr[i] = Layer(int(l.kind), float(l.pos), float(l.ext_lo), float(l.ext_hi),
                       float(l.var_u_max), float(l.var_v_max), int(l.n_phi_bins), int(l.n_q_bins),
                       float(getattr(l, "stereo", 0.0)), float(getattr(l, "hole_lo", 0.0)),
                       float(getattr(l, "hole_hi", 0.0)))
    return arr


class Context:
    """One library context bound to a HIP stream (torch's current stream
    unless given)."""

    def __init__(self, find_config, flags=0, stream=None):
        self.cfg = make_config(find_config, flags)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        self._stream = stream
        h = C.c_void_p()
        st = lib.mkf_create(C.byref(self.cfg), C.c_void_p(stream), C.byref(h))
        if st != MKF_OK:
            raise MkfError(st, lib.mkf_last_error(None).decode())
        self.h = h
        self._keep = []

    def close(self):
        if getattr(self, "h", None):
            lib.mkf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != MKF_OK:
            raise MkfError(st, lib.mkf_last_error(self.h).decode())

    def load_geometry(self, layers):
        self._check(lib.mkf_load_geometry(self.h, make_layers(layers), len(layers)))

    def load_steering(self, regions):
        """Region steering for the next seed(); an empty sequence returns to
        plans from each seed's helix."""
        self._check(lib.mkf_load_steering(self.h, make_regions(regions), len(regions)))

    def load_material(self, mm):
        """Material map (an object with n_r, n_z, r_max, z_max, mass, k_max
        and [n_z][n_r] tables x_x0, xi), or None for the constant angle."""
        if mm is None:
            self._check(lib.mkf_load_material(self.h, None, None, None))
            return
        info = MaterialInfo(int(mm.n_r), int(mm.n_z), float(mm.r_max), float(mm.z_max),
                            float(mm.mass), float(mm.k_max))
        t = np.ascontiguousarray(mm.x_x0, np.float32).reshape(-1)
        x = np.ascontiguousarray(mm.xi, np.float32).reshape(-1)
        if t.size != info.n_r * info.n_z or x.size != t.size:
            raise ValueError("material tables must hold n_z x n_r bins")
        self._check(lib.mkf_load_material(self.h, C.byref(info), t.ctypes.data, x.ctypes.data))

    def load_field(self, fd):
        """Parameterised field (an object with b0, c_r2, c_z2, c_z4, h_max), or
        None for the uniform field of the settings."""
        if fd is None:
            self._check(lib.mkf_load_field(self.h, None))
            return
        f = Field(float(fd.b0), float(fd.c_r2), float(fd.c_z2), float(fd.c_z4), float(fd.h_max))
        self._check(lib.mkf_load_field(self.h, C.byref(f)))

    def load_hits(self, ev_off, x, y, z, var_u, var_v, layer):
        ev_off = np.ascontiguousarray(ev_off, np.int64)
        arrs = (x, y, z, var_u, var_v, layer)
        dev = _is_device(x)
        assert all(_is_device(a) == dev for a in arrs)
        self._check(lib.mkf_load_hits(self.h, len(ev_off) - 1, _ptr(ev_off),
                                      *[_ptr(a) for a in arrs], MEM_DEVICE if dev else MEM_HOST))

    def seed(self, seed_event, seed_hits):
        dev = _is_device(seed_event)
        self._check(lib.mkf_seed(self.h, int(seed_event.shape[0]), _ptr(seed_event),
                                 _ptr(seed_hits), MEM_DEVICE if dev else MEM_HOST))

    def get_seed_states(self, n):
        par = np.zeros((n, 6), np.float32)
        cov = np.zeros((n, 21), np.float32)
        ok = np.zeros(n, np.int32)
        plen = np.zeros(n, np.int32)
        plan = np.zeros((n, MAX_PLAN), np.int8)
        chi2 = np.zeros(n, np.float32)
        self._check(lib.mkf_get_seed_states(self.h, _ptr(par), _ptr(cov), _ptr(ok), _ptr(plen),
                                            _ptr(plan), _ptr(chi2)))
        return par, cov, ok, plen, plan, chi2

    def find(self):
        self._check(lib.mkf_find(self.h))

    def get_tracks(self, n):
        out = np.zeros(n, TRACK_DTYPE)
        tot = C.c_int64()
        self._check(lib.mkf_get_tracks(self.h, _ptr(out), n, C.byref(tot)))
        return out

    def propagate(self, par, cov, layer, out_par, out_cov, out_l, out_status):
        self._check(lib.mkf_propagate(self.h, int(par.shape[0]), _ptr(par), _ptr(cov), _ptr(layer),
                                      _ptr(out_par), _ptr(out_cov), _ptr(out_l),
                                      _ptr(out_status)))

    def fit(self, kind, pos, x, y, z, var_u, var_v, length, init_par, init_cov, out_par,
            out_cov, out_chi2, out_status):
        n_steps, n = x.shape
        self._check(lib.mkf_fit(self.h, n, n_steps, _ptr(kind), _ptr(pos), _ptr(x), _ptr(y),
                                _ptr(z), _ptr(var_u), _ptr(var_v), _ptr(length), _ptr(init_par),
                                _ptr(init_cov), _ptr(out_par), _ptr(out_cov), _ptr(out_chi2),
                                _ptr(out_status)))

    def backward_fit(self, out_par, out_cov, out_chi2, out_status):
        """Backward fit of the last find's tracks into device arrays (seed
        order): out_par [n][6], out_cov [n][21], out_chi2 [n], out_status [n]."""
        self._check(lib.mkf_backward_fit(self.h, _ptr(out_par), _ptr(out_cov), _ptr(out_chi2),
                                         _ptr(out_status)))

    def smooth(self, out_par, out_cov, out_n):
        """Smoothed states of the last find's tracks into device arrays (seed
        order): out_par [n][MAX_PLAN + 1][6], out_cov [n][MAX_PLAN + 1][21],
        out_n [n] (surfaces per track)."""
        self._check(lib.mkf_smooth(self.h, _ptr(out_par), _ptr(out_cov), _ptr(out_n)))

    def make_seeds(self, seeding, capacity, out_event, out_hits):
        """Triplet seeds into device arrays out_event [capacity], out_hits
        [capacity][3]; returns their number (raises on MKF_E_CAPACITY, whose
        message holds the number needed)."""
        n = C.c_int64(0)
        st = lib.mkf_make_seeds(self.h, C.byref(make_seeding(seeding)), int(capacity),
                                _ptr(out_event), _ptr(out_hits), C.byref(n))
        if st == MKF_E_CAPACITY:
            raise MkfError(st, f"{n.value} triplets, capacity {capacity}")
        self._check(st)
        return int(n.value)

    def clean_seeds(self, cleaning, out_keep):
        """Seed cleaning of the loaded seeds into a device int32 array
        [n_seeds] (seed order, 1 = keep); returns the number kept."""
        cc = Cleaning(cleaning.tol_ipt, cleaning.tol_eta, cleaning.tol_phi)
        n = C.c_int64(0)
        self._check(lib.mkf_clean_seeds(self.h, C.byref(cc), _ptr(out_keep), C.byref(n)))
        return int(n.value)

    def find_duplicates(self, frac, out_dup):
        """Duplicate flags of the last find's tracks into a device int32
        array [n_seeds] (seed order); returns their number."""
        n = C.c_int64(0)
        self._check(lib.mkf_find_duplicates(self.h, float(frac), _ptr(out_dup), C.byref(n)))
        return int(n.value)

    def set_tuning(self, waves_per_simd, blocks_per_cu, lane_group=0, phi_bin_shift=0,
                   q_bin_shift=0):
        self._check(lib.mkf_set_tuning(self.h, C.byref(Tuning(waves_per_simd, blocks_per_cu,
                                                               lane_group, phi_bin_shift,
                                                               q_bin_shift))))

    def get_tuning(self):
        t = Tuning()
        self._check(lib.mkf_get_tuning(self.h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in Tuning._fields_}

    def autotune(self, repeats=2, cache_path=None):
        t = Tuning()
        self._check(lib.mkf_autotune(self.h, repeats,
                                     cache_path.encode() if cache_path else None, C.byref(t)))
        return {k: getattr(t, k) for k, _ in Tuning._fields_}

    # ---- learned propagation surrogate

    def surrogate_train(self, n_samples, epochs, batch, lr, seed, loss_w=(1, 0, 0, 0, 0, 0, 0),
                        first_step=0, n_steps=0):
        cfg = TrainCfg(int(n_samples), int(epochs), int(batch), float(lr), int(seed))
        for j in range(7):
            cfg.loss_w[j] = float(loss_w[j])
        cfg.first_step, cfg.n_steps = int(first_step), int(n_steps)
        rep = TrainReport()
        self._check(lib.mkf_surrogate_train(self.h, C.byref(cfg), C.byref(rep)))
        return {k: getattr(rep, k) for k, _ in TrainReport._fields_}

    def surrogate_get(self):
        out = np.zeros(MLP_NPARAM, np.float32)
        self._check(lib.mkf_surrogate_get(self.h, _ptr(out)))
        return out

    def surrogate_set(self, params):
        params = np.ascontiguousarray(params, np.float32)
        assert params.shape == (MLP_NPARAM,)
        self._check(lib.mkf_surrogate_set(self.h, _ptr(params)))

    def surrogate_save(self):
        """The training checkpoint as a byte blob (mkf_surrogate_save)."""
        n = C.c_size_t(0)
        st = lib.mkf_surrogate_save(self.h, None, 0, C.byref(n))
        assert st == MKF_E_CAPACITY, st
        buf = (C.c_ubyte * n.value)()
        self._check(lib.mkf_surrogate_save(self.h, buf, n.value, C.byref(n)))
        return bytes(buf)

    def surrogate_load(self, blob):
        blob = bytes(blob)
        buf = (C.c_ubyte * len(blob)).from_buffer_copy(blob)
        self._check(lib.mkf_surrogate_load(self.h, buf, len(blob)))

    def surrogate_get_state(self):
        """(params, m, v, step): the weights and Adam's state."""
        p, m, v = (np.zeros(MLP_NPARAM, np.float32) for _ in range(3))
        step = C.c_int32(0)
        self._check(lib.mkf_surrogate_get_state(self.h, _ptr(p), _ptr(m), _ptr(v),
                                                C.byref(step)))
        return p, m, v, int(step.value)

    def surrogate_set_state(self, params, m, v, step):
        arrs = [np.ascontiguousarray(a, np.float32) for a in (params, m, v)]
        for a in arrs:
            assert a.shape == (MLP_NPARAM,)
        self._check(lib.mkf_surrogate_set_state(self.h, *[_ptr(a) for a in arrs], int(step)))

    def surrogate_grad(self, x, t, loss_w):
        """x [n][8], t [n][7] device tensors; returns (grad, loss) on the host."""
        lw = np.ascontiguousarray(loss_w, np.float32)
        grad = np.zeros(MLP_NPARAM, np.float32)
        loss = np.zeros(1, np.float32)
        self._check(lib.mkf_surrogate_grad(self.h, int(x.shape[0]), _ptr(x), _ptr(t), _ptr(lw),
                                           _ptr(grad), _ptr(loss)))
        return grad, float(loss[0])

    def surrogate_grad_noalloc(self, x, t, loss_w, grad, loss):
        """Loss and gradient into device tensors grad [5191] and loss [1]
        without any device allocation (queued on the context's stream)."""
        lw = np.ascontiguousarray(loss_w, np.float32)
        self._check(lib.mkf_surrogate_grad_noalloc(self.h, int(x.shape[0]), _ptr(x), _ptr(t),
                                                   _ptr(lw), _ptr(grad), _ptr(loss)))

    def surrogate_infer(self, x, y):
        self._check(lib.mkf_surrogate_infer(self.h, int(x.shape[0]), _ptr(x), _ptr(y)))

    def surrogate_samples(self, n, seed, x, t, valid):
        self._check(lib.mkf_surrogate_samples(self.h, int(n), int(seed), _ptr(x), _ptr(t),
                                              _ptr(valid)))

    def stats(self):
        s = Stats()
        self._check(lib.mkf_get_stats(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}


def unpack_cov(c21):
    """Packed upper triangle (..., 21) -> full (..., 6, 6)."""
    c21 = np.asarray(c21)
    out = np.zeros(c21.shape[:-1] + (6, 6), c21.dtype)
    k = 0
    for i in range(6):
        for j in range(i, 6):
            out[..., i, j] = c21[..., k]
            out[..., j, i] = c21[..., k]
            k += 1
    return out


def pack_cov(full):
    full = np.asarray(full)
    idx = [(i, j) for i in range(6) for j in range(i, 6)]
    return np.stack([full[..., i, j] for i, j in idx], axis=-1)
