"""Fit-only stress inputs: many tracks, each crossing the same number of
layers of a random barrel or endcap geometry, with smeared hits (input side
only; the tracks come from the event generator's circle description).

Barrel tracks (|eta| < 1) cross n_layers cylinders at random radii in
4-100 cm; endcap tracks (1.8 < |eta| < 2.4) cross n_layers disks at random
|z| in 40-320 cm on their own side.  pT is log-uniform in 1-10 GeV/c, so
every track reaches every layer within its first half turn.  The fit starts
from the truth at the vertex, displaced by draws of its own prior
covariance, so the prior is consistent.
"""
from dataclasses import dataclass
from typing import Tuple

import numpy as np

from .events import _smear, event_rng, simulate_tracks
from .workloads import BARREL, DISK, EventRecipe, Layer

# prior of the fit: x, y, z (cm^2), q/pT relative (fraction^2), phi, theta (rad^2)
PRIOR_SIGMA = (0.01, 0.01, 0.1, 0.05, 1e-3, 1e-3)


def stress_geometry(n_layers: int, seed: int) -> Tuple[Tuple[Layer, ...], Tuple[Layer, ...]]:
    rng = event_rng(seed, 0xFFFF)
    radii = np.sort(rng.uniform(4.0, 100.0, n_layers))
    zs = np.sort(rng.uniform(40.0, 320.0, n_layers))
    barrel = tuple(Layer(BARREL, float(r), -500.0, 500.0, 9e-6, 1e-4) for r in radii)
    plus = tuple(Layer(DISK, float(z), 0.0, 200.0, 9e-6, 1e-4) for z in zs)
    return barrel, plus


@dataclass
class FitStress:
    kind: np.ndarray      # [n_steps][n] int8
    pos: np.ndarray       # [n_steps][n] float32 (radius or signed z)
    x: np.ndarray         # [n_steps][n] float32 hit coordinates
    y: np.ndarray
    z: np.ndarray
    var_u: np.ndarray     # [n_steps][n] float32
    var_v: np.ndarray
    length: np.ndarray    # [n] int32 (all n_steps)
    init_par: np.ndarray  # [n][6] float32
    init_cov: np.ndarray  # [n][21] float32 packed upper triangle
    truth: np.ndarray     # [n][6] float64 vertex truth


def _pack_diag(d):
    out = np.zeros((d.shape[0], 21))
    k = 0
    for i in range(6):
        out[:, k] = d[:, i]
        k += 6 - i
    return out


def _chunk(args):
    n, n_layers, seed, chunk, bz = args
    rng = event_rng(seed, chunk)
    barrel, plus = stress_geometry(n_layers, seed)
    is_end = rng.random(n) < 0.5
    side = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    eta = np.where(is_end, side * rng.uniform(1.8, 2.4, n), rng.uniform(-1.0, 1.0, n))
    pt = np.exp(rng.uniform(np.log(1.0), np.log(10.0), n))
    recipe = EventRecipe(pt_lo=1.0, pt_hi=10.0, sigma_vxy=0.005, sigma_vz=1.0)
    kind = np.zeros((n_layers, n), np.int8)
    pos = np.zeros((n_layers, n), np.float32)
    hits = np.zeros((5, n_layers, n), np.float32)
    init = np.zeros((n, 6))
    for sel, layers in [(np.nonzero(~is_end)[0], barrel),
                        (np.nonzero(is_end & (side > 0))[0], plus),
                        (np.nonzero(is_end & (side < 0))[0],
                         tuple(Layer(DISK, -l.pos, l.ext_lo, l.ext_hi, l.var_u_max, l.var_v_max)
                               for l in plus))]:
        if sel.size == 0:
            continue
        ini, trk, lay, st = simulate_tracks(rng, sel.size, list(layers), bz, recipe,
                                            pt=pt[sel], eta=eta[sel])
        init[sel] = ini
        hx, hy, hz, vu, vv = _smear(rng, list(layers), lay, st)
        order = np.lexsort((lay, trk))  # crossings are in layer order along each track
        trk, lay = trk[order], lay[order]
        counts = np.bincount(trk, minlength=sel.size)
        assert np.all(counts == n_layers), "a stress track missed a layer"
        col = sel[trk]
        step = np.tile(np.arange(n_layers), sel.size)
        kind[step, col] = layers[0].kind
        pos[step, col] = np.array([layers[k].pos for k in range(n_layers)])[lay]
        for a, v in enumerate((hx, hy, hz, vu, vv)):
            hits[a, step, col] = v[order]
    sig = np.array(PRIOR_SIGMA)[None, :] * np.ones((n, 1))
    sig[:, 3] *= np.abs(init[:, 3])
    par = init + rng.normal(size=(n, 6)) * sig
    return kind, pos, hits, par.astype(np.float32), _pack_diag(sig ** 2).astype(np.float32), init


def fit_stress(n_tracks: int, n_layers: int = 26, seed: int = 0x5EED0006, bz: float = 3.8,
               chunk: int = 65536, workers: int = 1) -> FitStress:
    jobs = [(min(chunk, n_tracks - c0), n_layers, seed, i, bz)
            for i, c0 in enumerate(range(0, n_tracks, chunk))]
    if workers > 1 and len(jobs) > 1:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(workers) as pool:
            parts = pool.map(_chunk, jobs)
    else:
        parts = [_chunk(j) for j in jobs]
    kind = np.concatenate([p[0] for p in parts], axis=1)
    pos = np.concatenate([p[1] for p in parts], axis=1)
    hits = np.concatenate([p[2] for p in parts], axis=2)
    return FitStress(kind, pos, hits[0], hits[1], hits[2], hits[3], hits[4],
                     np.full(n_tracks, n_layers, np.int32),
                     np.concatenate([p[3] for p in parts]), np.concatenate([p[4] for p in parts]),
                     np.concatenate([p[5] for p in parts]))
