"""Seeded synthetic event generator (input side only).

It simulates charged particles in a uniform solenoid field crossing the
layers of a workload geometry, records smeared hits, adds noise hits and
forms truth-matched seeds from each track's first three hits.  It describes
the truth and carries no part of the filter (no covariance, no chi2, no
Kalman update, no hit selection); its trajectory code is a separate
centre-and-angle description of the circle, independent of the oracle's and
the GPU library's propagation.

Random numbers come from numpy's Philox counter-based generator, keyed by
(workload master seed, event index), so every event is reproducible on its
own.
"""
from dataclasses import dataclass
from typing import List, Optional, Tuple

import numpy as np

from .workloads import BARREL, DISK, KAPPA, SIGMA_R, SIGMA_RPHI, SIGMA_Z, Workload


def event_rng(master_seed: int, event: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=(int(master_seed) << 32) | int(event)))


@dataclass
class Event:
    x: np.ndarray        # float32 hit coordinates
    y: np.ndarray
    z: np.ndarray
    var_u: np.ndarray    # float32 hit variances in the local frame
    var_v: np.ndarray
    layer: np.ndarray    # int32
    track: np.ndarray    # int32 truth track id, -1 for noise
    seeds: np.ndarray    # (n_seeds, 3) int32 event-local hit indices
    seed_track: np.ndarray  # int32 truth track of each seed
    # truth per recorded hit (float64): state after the layer at that hit
    # (position on the surface, q/pT, phi, theta after the scattering kick)
    truth_state: np.ndarray  # (n_hits, 6); NaN rows for noise
    track_hits: List[np.ndarray]  # per track: event-local hit indices in order
    # per track: the initial state (vertex, q/pT, phi, theta), float64
    track_init: Optional[np.ndarray] = None

    @property
    def n_hits(self) -> int:
        return int(self.x.shape[0])


def _wrap(a):
    return (a + np.pi) % (2.0 * np.pi) - np.pi


def _next_crossings(cx, cy, rho, sgn, x, y, z, cot, budget, kinds, poss, eps):
    """Transverse path length to the next crossing of every surface.

    The track is the circle of centre (cx, cy) and radius rho travelled with
    sense sgn (+1 anticlockwise); z rises by cot per unit transverse path.
    Returns an (n_tracks, n_surfaces) array, inf where there is no crossing
    within `budget` (the remaining transverse path of the half turn)."""
    n = x.shape[0]
    out = np.full((n, len(kinds)), np.inf)
    beta0 = np.arctan2(y - cy, x - cx)
    d = np.hypot(cx, cy)
    dhat_x, dhat_y = cx / d, cy / d
    for j, (kind, pos) in enumerate(zip(kinds, poss)):
        if kind == BARREL:
            R = pos
            # intersection of circle(centre, rho) with circle(origin, R):
            # the chord midpoint lies at distance a from the origin along
            # the centre direction, the chord half-length is hh
            a = (R * R - rho * rho + d * d) / (2.0 * d)
            hh2 = R * R - a * a
            ok = hh2 >= 0.0
            hh = np.sqrt(np.where(ok, hh2, 0.0))
            best = np.full(n, np.inf)
            for s in (1.0, -1.0):
                px = a * dhat_x - s * hh * dhat_y
                py = a * dhat_y + s * hh * dhat_x
                beta = np.arctan2(py - cy, px - cx)
                dturn = np.mod(sgn * (beta - beta0), 2.0 * np.pi)
                l = dturn * rho
                good = ok & (l > eps) & (l < budget)
                best = np.where(good & (l < best), l, best)
            out[:, j] = best
        else:
            Z = pos
            with np.errstate(divide="ignore", invalid="ignore"):
                l = (Z - z) / cot
            good = np.isfinite(l) & (l > eps) & (l < budget)
            out[:, j] = np.where(good, l, np.inf)
    return out


_ME = 0.51099895e-3      # electron mass, GeV
_K_BETHE = 0.307075e-3  # GeV cm^2 / mol
_SI_ZA, _SI_I = 0.49848, 173e-9


def _si_loss_rate(p, mass):
    """Mean ionisation loss rate in silicon, GeV cm^2/g, at momentum p
    (Bethe-Bloch without density effect)."""
    bg2 = (p / mass) ** 2
    g = np.sqrt(1.0 + bg2)
    b2 = bg2 / (1.0 + bg2)
    ratio = _ME / mass
    wmax = 2.0 * _ME * bg2 / (1.0 + 2.0 * g * ratio + ratio * ratio)
    return _K_BETHE * _SI_ZA / b2 * (0.5 * np.log(2.0 * _ME * bg2 * wmax / _SI_I ** 2) - b2)


def _material_kick(rng, mat, is_b, x, y, z, ph, th, p_tot):
    """Scattering angle (Highland, at the momentum before the loss) and
    mean ionisation loss of the material crossed at (x, y, z) by tracks of
    direction (ph, th) and momentum p_tot.  Returns (angle sigma, new p)."""
    r = np.hypot(x, y)
    ir = np.clip(np.floor(r / mat.r_max * mat.n_r).astype(int), 0, mat.n_r - 1)
    iz = np.clip(np.floor((z + mat.z_max) / (2.0 * mat.z_max) * mat.n_z).astype(int), 0,
                 mat.n_z - 1)
    t0 = np.asarray(mat.x_x0, np.float64)[iz, ir]
    xi0 = np.asarray(mat.xi, np.float64)[iz, ir]
    # incidence: track direction against the surface normal
    dx, dy, dz = np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)
    cos_in = np.where(is_b, (dx * x + dy * y) / r, dz)
    path = np.minimum(1.0 / np.maximum(np.abs(cos_in), 1e-300), mat.k_max)
    energy = np.sqrt(p_tot ** 2 + mat.mass ** 2)
    beta = p_tot / energy
    t = t0 * path
    with np.errstate(divide="ignore"):
        corr = np.maximum(1.0 + 0.038 * np.log(np.where(t > 0, t, 1.0)), 0.0)
    sigma = np.where(t > 0, 0.0136 / (beta * p_tot) * np.sqrt(t) * corr, 0.0)
    dp = np.minimum(xi0 * path * _si_loss_rate(p_tot, mat.mass) / beta, 0.5 * p_tot)
    return sigma, p_tot - np.where(xi0 > 0, dp, 0.0)


def _bz(field, x, y, z):
    r2, z2 = x * x + y * y, z * z
    return field.b0 * (1.0 + field.c_r2 * r2 + field.c_z2 * z2 + field.c_z4 * z2 * z2)


def _rk4(field, ipt, cot, x, y, z, ph, h):
    """One Runge-Kutta step of transverse length h (arrays) of the motion in
    the axial field: pT and theta constant, phi turning at -KAPPA Bz q/pT."""
    def d(x, y, z, ph):
        return np.cos(ph), np.sin(ph), cot, -KAPPA * _bz(field, x, y, z) * ipt
    k1 = d(x, y, z, ph)
    k2 = d(*(v + 0.5 * h * k for v, k in zip((x, y, z, ph), k1)))
    k3 = d(*(v + 0.5 * h * k for v, k in zip((x, y, z, ph), k2)))
    k4 = d(*(v + h * k for v, k in zip((x, y, z, ph), k3)))
    return tuple(v + h / 6.0 * (a + 2.0 * b + 2.0 * c + e)
                 for v, a, b, c, e in zip((x, y, z, ph), k1, k2, k3, k4))


def _simulate_field(rng, q, pt, theta, phi, vx, vy, vz, layers, recipe, field, material,
                    step=0.25):
    """Truth in a parameterised field: all tracks advance together in
    Runge-Kutta steps of `step` cm of transverse path; a step that crosses
    a layer is cut at the crossing (a disk's exactly, a barrel's by Newton
    iterations on the cut step), where the hit is recorded and the layer's
    scattering and loss applied.  A track stops after half a turn or when
    it leaves the detector."""
    n = q.shape[0]
    kinds = np.array([l.kind for l in layers])
    poss = np.array([l.pos for l in layers], float)
    lo = np.array([l.ext_lo for l in layers])
    hi = np.array([l.ext_hi for l in layers])
    is_b = kinds == BARREL
    r_out = max(max(poss[is_b], default=0.0), max(hi[~is_b], default=0.0)) + 5.0
    z_out = max(np.abs(poss[~is_b]).max(initial=0.0), np.abs(hi[is_b]).max(initial=0.0)) + 5.0
    x, y, z, ph = vx.copy(), vy.copy(), vz.copy(), phi.copy()
    th, ptc = theta.copy(), pt.copy()
    ph0 = phi.copy()
    alive = np.ones(n, bool)
    recs = []
    for _ in range(200000):
        idx = np.nonzero(alive)[0]
        if idx.size == 0:
            break
        ipt = q[idx] / ptc[idx]
        cot = np.cos(th[idx]) / np.sin(th[idx])
        x0, y0, z0, p0 = x[idx], y[idx], z[idx], ph[idx]
        x1, y1, z1, p1 = _rk4(field, ipt, cot, x0, y0, z0, p0, step)
        # fraction of the step to each layer's crossing (inf: none)
        frac = np.full((idx.size, len(layers)), np.inf)
        for k, L in enumerate(layers):
            if L.kind == BARREL:
                g0 = x0 * x0 + y0 * y0 - L.pos ** 2
                g1 = x1 * x1 + y1 * y1 - L.pos ** 2
                hit = (g0 != 0.0) & ((g0 < 0.0) != (g1 < 0.0))
                frac[hit, k] = (g0 / (g0 - g1))[hit]
            else:
                d0, d1 = z0 - L.pos, z1 - L.pos
                hit = (d0 != 0.0) & ((d0 < 0.0) != (d1 < 0.0))
                frac[hit, k] = (d0 / (d0 - d1))[hit]
        k = np.argmin(frac, axis=1)
        f = frac[np.arange(idx.size), k]
        cross = np.isfinite(f)
        # no crossing: take the whole step
        nc = ~cross
        x[idx[nc]], y[idx[nc]], z[idx[nc]], ph[idx[nc]] = x1[nc], y1[nc], z1[nc], p1[nc]
        if cross.any():
            c = np.nonzero(cross)[0]
            t = idx[c]
            kk = k[c]
            s = f[c] * step
            bar = is_b[kk]
            # disks: z is linear in the path, so the fraction is exact;
            # barrels: Newton on the cut step length
            for _it in range(4):
                xs, ys, zs, ps = _rk4(field, ipt[c], cot[c], x0[c], y0[c], z0[c], p0[c], s)
                g = xs * xs + ys * ys - poss[kk] ** 2
                gp = 2.0 * (xs * np.cos(ps) + ys * np.sin(ps))
                s = np.where(bar & (gp != 0.0), s - g / np.where(gp != 0.0, gp, 1.0), s)
            xs, ys, zs, ps = _rk4(field, ipt[c], cot[c], x0[c], y0[c], z0[c], p0[c], s)
            rr = np.hypot(xs, ys)
            xs = np.where(bar, xs * poss[kk] / rr, xs)
            ys = np.where(bar, ys * poss[kk] / rr, ys)
            zs = np.where(bar, zs, poss[kk])
            # step just past the surface so that it is not found again
            x[t], y[t], z[t], ph[t] = xs, ys, zs, ps
            qv = np.where(bar, zs, np.hypot(xs, ys))
            inside = (qv >= lo[kk]) & (qv <= hi[kk])
            sel = np.nonzero(inside)[0]
            if sel.size:
                tt = t[sel]
                if material is not None:
                    p_tot = ptc[tt] / np.sin(th[tt])
                    sig, p_new = _material_kick(rng, material, bar[sel], x[tt], y[tt], z[tt],
                                                ph[tt], th[tt], p_tot)
                    dth = rng.normal(0.0, 1.0, tt.size) * sig
                    dal = rng.normal(0.0, 1.0, tt.size) * sig
                    ph[tt] = ph[tt] + dal / np.sin(th[tt])
                    th[tt] = th[tt] + dth
                    ptc[tt] = p_new * np.sin(th[tt])
                elif recipe.ms_sigma > 0.0:
                    dth = rng.normal(0.0, recipe.ms_sigma, tt.size)
                    dal = rng.normal(0.0, recipe.ms_sigma, tt.size)
                    p_tot = ptc[tt] / np.sin(th[tt])
                    ph[tt] = ph[tt] + dal / np.sin(th[tt])
                    th[tt] = th[tt] + dth
                    ptc[tt] = p_tot * np.sin(th[tt])
                state = np.stack([x[tt], y[tt], z[tt], q[tt] / ptc[tt], _wrap(ph[tt]), th[tt]],
                                 axis=1)
                recs.append((tt, kk[sel].astype(np.int32), state))
            # nudge past the surface along the direction
            x[t] += 1e-7 * np.cos(ph[t])
            y[t] += 1e-7 * np.sin(ph[t])
            z[t] += 1e-7 * np.cos(th[t]) / np.sin(th[t])
        gone = ((np.abs(ph[idx] - ph0[idx]) >= np.pi) | (np.hypot(x[idx], y[idx]) > r_out) |
                (np.abs(z[idx]) > z_out))
        alive[idx[gone]] = False
    if recs:
        return (np.concatenate([r[0] for r in recs]), np.concatenate([r[1] for r in recs]),
                np.concatenate([r[2] for r in recs]))
    return np.zeros(0, np.int64), np.zeros(0, np.int32), np.zeros((0, 6))


def simulate_tracks(rng, n, layers, bz, recipe, pt=None, eta=None, phi=None, q=None,
                    vertex=None, max_iter=64, material=None, field=None):
    """Simulate n tracks; returns per-crossing records (track, layer, true
    position, state after the layer) in crossing order, plus the initial
    parameters.  With a material map, each crossed layer scatters the track
    by the Highland angle of its material and takes its mean ionisation
    loss (in place of the recipe's constant angle)."""
    if q is None:
        q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    if pt is None:
        pt = np.exp(rng.uniform(np.log(recipe.pt_lo), np.log(recipe.pt_hi), n))
    if eta is None:
        eta = rng.uniform(-recipe.eta_max, recipe.eta_max, n)
    if phi is None:
        phi = rng.uniform(-np.pi, np.pi, n)
    if vertex is None:
        vx = rng.normal(0.0, recipe.sigma_vxy, n)
        vy = rng.normal(0.0, recipe.sigma_vxy, n)
        vz = rng.normal(0.0, recipe.sigma_vz, n)
    else:
        vx, vy, vz = vertex
    theta = 2.0 * np.arctan(np.exp(-eta))
    init = np.stack([vx, vy, vz, q / pt, phi, theta], axis=1)
    if field is not None:
        trk, lay, st = _simulate_field(rng, q, pt, theta, phi, vx, vy, vz, layers, recipe, field,
                                       material)
        return init, trk, lay, st

    kinds = [l.kind for l in layers]
    poss = [l.pos for l in layers]
    x, y, z = vx.copy(), vy.copy(), vz.copy()
    ph, th, ptc = phi.copy(), theta.copy(), pt.copy()
    turned = np.zeros(n)          # transverse turning angle so far
    alive = np.ones(n, bool)
    eps = 1e-6
    recs = []
    for _ in range(max_iter):
        idx = np.nonzero(alive)[0]
        if idx.size == 0:
            break
        omega = -KAPPA * bz * q[idx] / ptc[idx]      # signed curvature
        rho = 1.0 / np.abs(omega)
        sgn = np.sign(omega)
        # centre: a quarter turn from the direction, toward the turning side
        cx = x[idx] - np.sin(ph[idx]) / omega
        cy = y[idx] + np.cos(ph[idx]) / omega
        cot = np.cos(th[idx]) / np.sin(th[idx])
        budget = (np.pi - turned[idx]) * rho
        L = _next_crossings(cx, cy, rho, sgn, x[idx], y[idx], z[idx], cot, budget,
                            kinds, poss, eps)
        j = np.argmin(L, axis=1)
        l = L[np.arange(idx.size), j]
        done = ~np.isfinite(l)
        alive[idx[done]] = False
        keep = ~done
        idx, j, l = idx[keep], j[keep], l[keep]
        omega, cx, cy, cot, rho = omega[keep], cx[keep], cy[keep], cot[keep], rho[keep]
        if idx.size == 0:
            break
        beta0 = np.arctan2(y[idx] - cy, x[idx] - cx)
        beta = beta0 + omega * l
        nx = cx + rho * np.cos(beta)
        ny = cy + rho * np.sin(beta)
        nz = z[idx] + l * cot
        # the layer's tangent-plane definition puts a barrel crossing on r = R
        # and a disk crossing on z = Z exactly
        is_b = np.array([kinds[k] == BARREL for k in j])
        posj = np.array([poss[k] for k in j])
        rr = np.hypot(nx, ny)
        nx = np.where(is_b, nx * posj / rr, nx)
        ny = np.where(is_b, ny * posj / rr, ny)
        nz = np.where(is_b, nz, posj)
        x[idx], y[idx], z[idx] = nx, ny, nz
        ph[idx] = _wrap(ph[idx] + omega * l)
        turned[idx] += np.abs(omega) * l
        lo = np.array([layers[k].ext_lo for k in j])
        hi = np.array([layers[k].ext_hi for k in j])
        qv = np.where(is_b, nz, np.hypot(nx, ny))
        inside = (qv >= lo) & (qv <= hi)
        sel = np.nonzero(inside)[0]
        if sel.size:
            t = idx[sel]
            # scattering on the crossed layer, after the hit is made
            if material is not None:
                p_tot = ptc[t] / np.sin(th[t])
                sig, p_new = _material_kick(rng, material, is_b[sel], x[t], y[t], z[t], ph[t],
                                            th[t], p_tot)
                dth = rng.normal(0.0, 1.0, t.size) * sig
                dal = rng.normal(0.0, 1.0, t.size) * sig
                ph[t] = _wrap(ph[t] + dal / np.sin(th[t]))
                th[t] = th[t] + dth
                ptc[t] = p_new * np.sin(th[t])
            elif recipe.ms_sigma > 0.0:
                dth = rng.normal(0.0, recipe.ms_sigma, t.size)
                dal = rng.normal(0.0, recipe.ms_sigma, t.size)
                p_tot = ptc[t] / np.sin(th[t])
                ph[t] = _wrap(ph[t] + dal / np.sin(th[t]))
                th[t] = th[t] + dth
                ptc[t] = p_tot * np.sin(th[t])
            state = np.stack([x[t], y[t], z[t], q[t] / ptc[t], ph[t], th[t]], axis=1)
            recs.append((t, j[sel], state))
    if recs:
        trk = np.concatenate([r[0] for r in recs])
        lay = np.concatenate([r[1] for r in recs]).astype(np.int32)
        st = np.concatenate([r[2] for r in recs])
    else:
        trk = np.zeros(0, np.int64)
        lay = np.zeros(0, np.int32)
        st = np.zeros((0, 6))
    return init, trk, lay, st


def _smear(rng, layers, lay, st):
    """Smeared hit positions on their layer surfaces and their variances
    (along and across the strips; on a layer without stereo angle these are
    u = r-phi and v = z or r)."""
    n = lay.shape[0]
    kind = np.array([layers[k].kind for k in lay]) if n else np.zeros(0, int)
    posv = np.array([layers[k].pos for k in lay]) if n else np.zeros(0)
    x, y, z = st[:, 0], st[:, 1], st[:, 2]
    r = np.hypot(x, y)
    phi = np.arctan2(y, x)
    e_u = rng.normal(0.0, SIGMA_RPHI, n)
    e_v = rng.normal(0.0, 1.0, n)
    is_b = kind == BARREL
    sig_v = np.where(is_b, SIGMA_Z, SIGMA_R)
    du, dv = e_u, e_v * sig_v
    vu = np.full(n, SIGMA_RPHI ** 2)
    vv = sig_v ** 2
    stereo = np.array([layers[k].stereo for k in lay]) if n else np.zeros(0)
    st_m = stereo != 0.0
    if np.any(st_m):
        # strips turned by a: the error e_u lies along w = (cos a, sin a) in
        # (u, v), the error across them (sigma_perp) along (-sin a, cos a)
        sp = np.array([layers[k].sigma_perp for k in lay])
        c, s = np.cos(stereo), np.sin(stereo)
        ep = e_v * sp
        du = np.where(st_m, c * e_u - s * ep, du)
        dv = np.where(st_m, s * e_u + c * ep, dv)
        vv = np.where(st_m, sp ** 2, vv)
    # barrel: along the cylinder in r-phi, and in z; disk: r-phi and r
    rb = np.where(is_b, posv, r + dv)
    phib = phi + du / np.where(is_b, posv, r)
    hx = rb * np.cos(phib)
    hy = rb * np.sin(phib)
    hz = np.where(is_b, z + dv, posv)
    return hx, hy, hz, vu, vv


def _noise(rng, layers, counts, frac):
    xs, ys, zs, vus, vvs, ls = [], [], [], [], [], []
    for k, layer in enumerate(layers):
        m = int(round(frac * counts[k]))
        if m == 0:
            continue
        phi = rng.uniform(-np.pi, np.pi, m)
        if layer.kind == BARREL:
            r = np.full(m, layer.pos)
            z = rng.uniform(layer.ext_lo, layer.ext_hi, m)
            vv = np.full(m, SIGMA_Z ** 2)
        else:
            r = np.sqrt(rng.uniform(layer.ext_lo ** 2, layer.ext_hi ** 2, m))
            z = np.full(m, layer.pos)
            vv = np.full(m, SIGMA_R ** 2)
        if layer.stereo != 0.0:
            vv = np.full(m, layer.sigma_perp ** 2)
        if layer.hole_lo < layer.hole_hi:
            q = z if layer.kind == BARREL else r
            keep = ~((q > layer.hole_lo) & (q < layer.hole_hi))
            phi, r, z, vv = phi[keep], r[keep], z[keep], vv[keep]
            m = int(keep.sum())
        xs.append(r * np.cos(phi))
        ys.append(r * np.sin(phi))
        zs.append(z)
        vus.append(np.full(m, SIGMA_RPHI ** 2))
        vvs.append(vv)
        ls.append(np.full(m, k, np.int32))
    if not xs:
        e = np.zeros(0)
        return e, e, e, e, e, np.zeros(0, np.int32)
    return (np.concatenate(xs), np.concatenate(ys), np.concatenate(zs),
            np.concatenate(vus), np.concatenate(vvs), np.concatenate(ls))


def generate_event(w: Workload, event: int, n_tracks: Optional[int] = None,
                   phi_range: Optional[Tuple[float, float]] = None) -> Event:
    """One seeded event.  phi_range confines the tracks' initial azimuth (a
    dense, jet-like event: the hit density of many more tracks in a sector,
    at the cost of few)."""
    rng = event_rng(w.master_seed, event)
    lo, hi = w.n_tracks
    if n_tracks is None:
        n_tracks = lo if lo == hi else int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
    phi = None if phi_range is None else rng.uniform(phi_range[0], phi_range[1], n_tracks)
    init, trk, lay, st = simulate_tracks(rng, n_tracks, w.layers, w.find.bz, w.recipe, phi=phi,
                                         material=w.material, field=w.field)
    # 2% (or as configured) independent loss of hits
    if w.recipe.hit_ineff > 0.0:
        keep = rng.random(trk.shape[0]) >= w.recipe.hit_ineff
        trk, lay, st = trk[keep], lay[keep], st[keep]
    # crossings inside a layer's hole leave no hit
    if any(L.hole_lo < L.hole_hi for L in w.layers):
        hl = np.array([L.hole_lo for L in w.layers])[lay]
        hh = np.array([L.hole_hi for L in w.layers])[lay]
        isb = np.array([L.kind == BARREL for L in w.layers])[lay]
        q = np.where(isb, st[:, 2], np.hypot(st[:, 0], st[:, 1]))
        keep = ~((q > hl) & (q < hh))
        trk, lay, st = trk[keep], lay[keep], st[keep]
    hx, hy, hz, vu, vv = _smear(rng, w.layers, lay, st)
    counts = np.bincount(lay, minlength=len(w.layers))
    nx, ny, nz, nvu, nvv, nl = _noise(rng, w.layers, counts, w.recipe.noise_frac)
    X = np.concatenate([hx, nx]).astype(np.float32)
    Y = np.concatenate([hy, ny]).astype(np.float32)
    Zc = np.concatenate([hz, nz]).astype(np.float32)
    VU = np.concatenate([vu, nvu]).astype(np.float32)
    VV = np.concatenate([vv, nvv]).astype(np.float32)
    LAY = np.concatenate([lay, nl]).astype(np.int32)
    TRK = np.concatenate([trk, np.full(nl.shape[0], -1)]).astype(np.int32)
    TS = np.concatenate([st, np.full((nl.shape[0], 6), np.nan)])
    # hits in random order: nothing may depend on the input order
    perm = rng.permutation(X.shape[0])
    X, Y, Zc, VU, VV, LAY, TRK, TS = (a[perm] for a in (X, Y, Zc, VU, VV, LAY, TRK, TS))
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.shape[0])
    # per-track hit lists in crossing order (records were made in order)
    n_true = trk.shape[0]
    new_idx = inv[:n_true]
    order = np.argsort(trk, kind="stable")
    bounds = np.searchsorted(trk[order], np.arange(n_tracks + 1))
    track_hits = [new_idx[order[bounds[t]:bounds[t + 1]]].astype(np.int32)
                  for t in range(n_tracks)]
    seeds, seed_track = [], []
    for t, h in enumerate(track_hits):
        if h.shape[0] >= 3:
            seeds.append(h[:3])
            seed_track.append(t)
    seeds = np.array(seeds, np.int32).reshape(-1, 3)
    return Event(X, Y, Zc, VU, VV, LAY, TRK, seeds, np.array(seed_track, np.int32),
                 TS, track_hits, init)


@dataclass
class EventBatch:
    """Several events concatenated: hits of event e are
    [ev_off[e], ev_off[e+1]); seeds carry their event and event-local
    hit indices."""
    ev_off: np.ndarray      # int64 (n_events + 1)
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    var_u: np.ndarray
    var_v: np.ndarray
    layer: np.ndarray
    seed_event: np.ndarray  # int32
    seed_hits: np.ndarray   # (n_seeds, 3) int32, event-local
    events: List[Event]

    @property
    def n_events(self) -> int:
        return len(self.events)


def make_batch(events: List[Event]) -> EventBatch:
    off = np.zeros(len(events) + 1, np.int64)
    off[1:] = np.cumsum([e.n_hits for e in events])
    cat = lambda f: np.concatenate([getattr(e, f) for e in events])
    se = np.concatenate([np.full(e.seeds.shape[0], i, np.int32) for i, e in enumerate(events)])
    sh = np.concatenate([e.seeds for e in events]).astype(np.int32).reshape(-1, 3)
    return EventBatch(off, cat("x"), cat("y"), cat("z"), cat("var_u"), cat("var_v"),
                      cat("layer"), se, sh, events)


def _gen_one(args):
    return generate_event(*args)


def generate(w: Workload, events=None, workers: int = 1) -> EventBatch:
    """Events of a workload (all by default).  workers > 1 generates them in
    that many spawned processes; every event depends only on its own key, so
    the result is the same."""
    if events is None:
        events = range(w.n_events)
    events = list(events)
    if workers > 1 and len(events) > 1:
        import multiprocessing as mp
        pool = mp.get_context("spawn").Pool(workers)
        try:
            evs = pool.map(_gen_one, [(w, e) for e in events], chunksize=1)
        finally:
            # let the workers exit on their own (no terminate signal)
            pool.close()
            pool.join()
    else:
        evs = [generate_event(w, e) for e in events]
    return make_batch(evs)
