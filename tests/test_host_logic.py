"""Host-side logic (CPU): the parity metric's handling of a surface's pinned
direction, the fit-stress input generator, and the surrogate's training
targets as functions of its rotation-invariant inputs."""
import numpy as np
import pytest

import parity as PT
from oracle import oracle as O
from synth import FindConfig
from synth.fitstress import PRIOR_SIGMA, fit_stress


def random_psd(rng, n=6):
    A = rng.normal(size=(n, n))
    return A @ A.T + n * np.eye(n)


def test_cov_err_is_zero_for_equal_and_scales_as_correlation():
    rng = np.random.default_rng(1)
    C = random_psd(rng)
    assert PT.cov_err(C, C) == 0.0
    D = C.copy()
    D[1, 2] = D[2, 1] = C[1, 2] + 0.01 * np.sqrt(C[1, 1] * C[2, 2])
    assert PT.cov_err(D, C) == pytest.approx(0.01, rel=1e-9)


def test_cov_err_ignores_the_pinned_normal_direction():
    """A covariance whose position block has a zero-variance direction (a
    state on a surface): a perturbation only along that direction is not
    an error, one in the free coordinates is."""
    rng = np.random.default_rng(2)
    C = random_psd(rng)
    n = np.array([0.6, 0.8, 0.0])  # barrel normal at azimuth 53 degrees
    P = np.eye(6)
    P[:3, :3] -= np.outer(n, n)
    C = P @ C @ P.T                # n^T C n = 0
    N = np.zeros(6)
    N[:3] = n
    noisy = C + 1e-9 * np.trace(C) * np.outer(N, N)
    assert PT.cov_err(noisy, C) < 1e-12
    bad = C.copy()
    bad[3, 3] *= 1.01
    assert PT.cov_err(bad, C) == pytest.approx(0.01, rel=1e-6)


def test_fit_stress_tracks_cross_every_layer_and_fit_with_consistent_prior():
    """Every generated track has one hit per layer, in increasing path
    order, and the oracle's fit through them gives chi2 per degree of
    freedom near one (the prior draws and hit smearing match the fit's
    model; the model's scattering term, absent from the truth, only lowers
    it)."""
    f = fit_stress(400, 12, seed=7)
    k, n = f.x.shape
    assert (k, n) == (12, 400)
    r = np.hypot(f.x, f.y)
    barrel = f.kind[0] == 0
    assert np.all(np.diff(r[:, barrel], axis=0) > 0)
    assert np.all(np.diff(np.abs(f.z[:, ~barrel]), axis=0) > 0)
    fc = FindConfig(ms_sigma=0.0)
    chi2 = []
    for t in range(0, n, 4):
        C0 = np.zeros((6, 6))
        k_ = 0
        for i in range(6):
            for j in range(i, 6):
                C0[i, j] = C0[j, i] = f.init_cov[t, k_]
                k_ += 1
        rc, p, C, c2 = O.fit_track(fc, f.init_par[t].astype(float), C0, f.kind[:, t].astype(np.int32),
                                   f.pos[:, t].astype(float),
                                   np.stack([f.x[:, t], f.y[:, t], f.z[:, t]], 1).astype(float),
                                   f.var_u[:, t].astype(float), f.var_v[:, t].astype(float))
        assert rc == 0
        chi2.append(c2)
    ndf = 2 * k
    assert 0.8 < np.mean(chi2) / ndf < 1.2
    assert len(PRIOR_SIGMA) == 6


def test_surrogate_target_is_invariant_under_rotation():
    """The network sees r0/R, the angle between direction and radius, omega R
    and the longitudinal terms: rotating a state about z must leave the
    crossing path, hence the first target, unchanged."""
    fc = FindConfig()
    rng = np.random.default_rng(3)
    for _ in range(20):
        R0, R1 = 25.0, 34.0
        a0 = rng.uniform(-np.pi, np.pi)
        p = np.array([R0 * np.cos(a0), R0 * np.sin(a0), rng.uniform(-20, 20),
                      rng.choice([-1, 1]) / rng.uniform(0.5, 10), a0 + rng.uniform(-0.3, 0.3),
                      rng.uniform(0.5, 2.6)])
        l = O.path_to_barrel(p, R1, fc.bz, fc.kappa, fc.l_min)
        rot = rng.uniform(-np.pi, np.pi)
        c, s = np.cos(rot), np.sin(rot)
        q = p.copy()
        q[0], q[1] = c * p[0] - s * p[1], s * p[0] + c * p[1]
        q[4] = (p[4] + rot + np.pi) % (2 * np.pi) - np.pi
        lq = O.path_to_barrel(q, R1, fc.bz, fc.kappa, fc.l_min)
        assert l == pytest.approx(lq, rel=1e-12)
