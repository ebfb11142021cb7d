"""Parity helpers: compare the GPU path with the FP64 oracle.

Tolerances (the arithmetic is FP32 on the GPU, FP64 in the oracle):
  parameters: |d| <= 1e-4 * max(|ref|, s) with s = the radial position scale
              for x, y, z, |q/pT| for q/pT, 1 rad for phi and theta;
  chi2:       |d| <= 1e-3 * chi2 + 1e-2 (the absolute floor covers FP32
              rounding of positions near 100 cm, ~1e-3 of a 30 um hit error);
  indices:    equal, unless the oracle flagged a decision of that seed as
              lying within the chi2 tolerance of the cut or of a tie, or an
              extent decision within 1e-3 cm of a widened edge; then the
              GPU's track must agree with the oracle up to the first such
              decision and be a valid path beyond it (explain_mismatch).
"""
import numpy as np

from oracle import oracle as O

PAR_REL = 1e-4
CHI2_REL, CHI2_ABS = 1e-3, 1e-2
# Covariance after ~10-25 chained FP32 propagations and Joseph-form updates,
# in units of sqrt(C_ii C_jj) in the surface's five free coordinates: the
# measured worst cases are 5e-4 (found tracks) and 8e-4 (fits of 3,000
# tracks through up to 14 hits); the bound leaves a factor 6.
COV_REL_FOUND = 5e-3
# A track that meets a layer almost tangentially (cosine between direction
# and surface normal below 0.2) makes the surface projection divide by that
# cosine, and FP32 cancels terms ~1/cos^2 larger than the result (a
# 0.40 GeV/c track reaching R = 70 cm has cos = 0.075).  With the Joseph-form
# update the measured worst case over 149 such fits is 0.018 on the GPU (0.073
# in a host build of the same arithmetic with other rounding of the
# transcendentals); the gain form reached 0.9 on the GPU and 31 on the host.
GRAZING_COS = 0.2
COV_REL_GRAZING = 0.1


def wrap(a):
    return (a + np.pi) % (2 * np.pi) - np.pi


def par_ok(g, r):
    g = np.asarray(g, np.float64)
    r = np.asarray(r, np.float64)
    spos = max(np.hypot(r[0], r[1]), abs(r[2]), 1.0)
    d = g - r
    d[4] = wrap(d[4])
    scale = np.array([max(abs(r[0]), spos), max(abs(r[1]), spos), max(abs(r[2]), spos),
                      abs(r[3]), 1.0, 1.0])
    return bool(np.all(np.abs(d) <= PAR_REL * scale)), d / scale


def cov_err(g, r):
    """Largest |dC_ij| / sqrt(C_ii C_jj) (the error in correlation units).

    A state on a surface has a pinned direction: the surface normal, in
    which the reference covariance has (numerically) zero variance.  Its
    entries there only carry FP32 rounding of the other entries, so when
    the reference's 3x3 position block has such a direction (variance below
    1e-8 of the largest) both covariances are compared in the remaining
    five coordinates."""
    g = np.asarray(g, np.float64)
    r = np.asarray(r, np.float64)
    w, V = np.linalg.eigh(r[:3, :3])
    if w[-1] > 0 and w[0] <= 1e-8 * w[-1]:
        J = np.zeros((5, 6))
        J[0, :3] = V[:, 1]
        J[1, :3] = V[:, 2]
        J[2, 3] = J[3, 4] = J[4, 5] = 1.0
        g = J @ g @ J.T
        r = J @ r @ J.T
    d = np.abs(np.diag(r))
    dg = np.sqrt(np.maximum(d, 1e-10 * d.max()))
    scale = np.outer(dg, dg)
    return float((np.abs(g - r) / scale).max())


def cov_ok(g, r, rel=2e-3):
    """Covariances: each entry within rel of sqrt(C_ii C_jj)."""
    return cov_err(g, r) <= rel


def chi2_ok(g, r):
    return abs(float(g) - float(r)) <= CHI2_REL * abs(float(r)) + CHI2_ABS


def explain_mismatch(g, r):
    """Whether the GPU's hit list g may differ from the oracle's result r.
    Before the oracle's first fragile step f every
    decision is clear, so the GPU's candidates there are the oracle's: its
    track's first f entries must be the history of a candidate the oracle
    had alive at step f (kept or retired).  From f on, its decisions must
    each be valid (the oracle follows its history: hits below the cut
    within tolerance, misses with a hole left, skips without a crossing,
    retiring with nothing compatible), and its hit count and chi2 must be
    the ones that path gives.  If only the final choice was fragile, the
    two results must tie in (hits, chi2).  Returns (first differing step,
    f) when excused, or a string saying what failed."""
    n = len(r["plan"])
    gh = [int(v) for v in g["hit"][:n]]
    rh = [int(v) for v in r["hit"]]
    d = next((k for k in range(n) if gh[k] != rh[k]), n)
    f = int(r["fragile_step"])
    if f < 0:
        return f"no fragile decision (first difference at step {d})"
    if f > 0:
        pre = O.find_prefixes(r, f)
        if not any(list(p[:f]) == gh[:f] for p in pre):
            return f"differs before the first fragile step {f} (at step {d})"
    st, path = O.follow_path(r, gh)
    if st != 0:
        return f"invalid decision at step {path['bad_step']} (status {st})"
    if path["n_hits"] != int(g["n_hits"]) or not chi2_ok(g["chi2"], path["chi2"]):
        return (f"path totals: GPU {int(g['n_hits'])} hits chi2 {float(g['chi2'])}, "
                f"the path gives {path['n_hits']} hits chi2 {path['chi2']}")
    if f >= n and (int(g["n_hits"]) != r["n_hits"] or not chi2_ok(g["chi2"], r["chi2"])):
        return "only the final choice was fragile, but the results do not tie"
    return (d, f)


def compare_tracks(gpu, ref, full_cov, cov_rel=COV_REL_FOUND):
    """gpu: records (TRACK_DTYPE) of the sampled seeds; ref: oracle dicts.
    Returns counts; 'fail' lists unexplained mismatches, 'diverged' the
    (sample index, first differing step, first fragile step) of the
    excused ones."""
    out = {"n": 0, "equal": 0, "tie_diverged": 0, "plan_diverged": 0, "fragile": 0,
           "max_cov_err": 0.0, "fail": [], "diverged": []}
    for i, (g, r) in enumerate(zip(gpu, ref)):
        out["n"] += 1
        fragile = r["fragile_step"] >= 0
        out["fragile"] += fragile
        if not r["seed_ok"]:
            if g["status"] != 0:
                out["fail"].append((i, "seed ok on GPU only"))
            continue
        if g["status"] != 1:
            out["fail"].append((i, "seed failed on GPU only"))
            continue
        n = len(r["plan"])
        if g["plan_len"] != n or list(g["plan"][:n]) != list(r["plan"]):
            if r["plan_fragile"]:
                out["plan_diverged"] += 1
            else:
                out["fail"].append((i, "plan", list(g["plan"][:g["plan_len"]]), list(r["plan"])))
            continue
        same = list(g["hit"][:n]) == list(r["hit"]) and g["n_hits"] == r["n_hits"]
        if not same:
            why = explain_mismatch(g, r)
            if isinstance(why, tuple):
                out["tie_diverged"] += 1
                out["diverged"].append((i,) + why)
            else:
                out["fail"].append((i, "hits", why, list(g["hit"][:n]), list(r["hit"])))
            continue
        ok_p, rel = par_ok(g["par"], r["par"])
        ok_c = chi2_ok(g["chi2"], r["chi2"])
        ce = cov_err(full_cov(g["cov"]), r["cov"])
        out["max_cov_err"] = max(out["max_cov_err"], ce)
        ok_v = ce <= cov_rel
        if ok_p and ok_c and ok_v:
            out["equal"] += 1
        else:  # same hits, same arithmetic: no excuse
            out["fail"].append((i, "numeric", ok_p, ok_c, ok_v, rel.tolist(),
                                float(g["chi2"]), float(r["chi2"])))
    return out


def conditioning(w, ev, hits):
    """Smallest cosine between the true direction and the surface normal
    over the track's hits (noise hits have no truth and are left out)."""
    cmin = 1.0
    for i in hits:
        s = ev.truth_state[i]
        if not np.all(np.isfinite(s)):
            continue
        d = np.array([np.cos(s[4]), np.sin(s[4]), 1 / np.tan(s[5])])
        nrm = (np.array([s[0], s[1], 0.0]) if w.layers[ev.layer[i]].kind == 0
               else np.array([0.0, 0.0, 1.0]))
        cmin = min(cmin, abs(d @ nrm) / np.linalg.norm(d) / np.linalg.norm(nrm))
    return cmin
