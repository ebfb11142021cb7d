"""Independent helix references used to pin the oracle (test code only).

None of this shares code with the oracle: it integrates the Lorentz force
with classical RK4, describes the circle by its centre and turning angle, and
finds surface crossings by dense sampling plus bisection.
"""
import numpy as np

KAPPA = 0.299792458e-2


def rk4_track(p, s_total, bz, kappa=KAPPA, n_steps=20000):
    """Integrate d r/ds = u, d u/ds = (kappa q B / |p|) u x z_hat over the 3-D
    path s_total.  p = (x, y, z, q/pT, phi, theta).  Returns (r, u)."""
    x, y, z, ipt, phi, th = p
    q = np.sign(ipt)
    pmag = 1.0 / (abs(ipt) * np.sin(th))
    r = np.array([x, y, z], float)
    u = np.array([np.cos(phi) * np.sin(th), np.sin(phi) * np.sin(th), np.cos(th)])
    c = kappa * q * bz / pmag
    bhat = np.array([0.0, 0.0, 1.0])

    def f(r_, u_):
        return u_, c * np.cross(u_, bhat)

    h = s_total / n_steps
    for _ in range(n_steps):
        k1r, k1u = f(r, u)
        k2r, k2u = f(r + 0.5 * h * k1r, u + 0.5 * h * k1u)
        k3r, k3u = f(r + 0.5 * h * k2r, u + 0.5 * h * k2u)
        k4r, k4u = f(r + h * k3r, u + h * k3u)
        r = r + h / 6.0 * (k1r + 2 * k2r + 2 * k3r + k4r)
        u = u + h / 6.0 * (k1u + 2 * k2u + 2 * k3u + k4u)
    return r, u


def centre_form(p, l, bz, kappa=KAPPA):
    """State after transverse path l using the circle centre and the turning
    angle (valid for B != 0)."""
    x, y, z, ipt, phi, th = p
    w = -kappa * bz * ipt
    cx, cy = x - np.sin(phi) / w, y + np.cos(phi) / w
    ang = phi + w * l
    return np.array([cx + np.sin(ang) / w, cy - np.cos(ang) / w,
                     z + l / np.tan(th), ipt, np.arctan2(np.sin(ang), np.cos(ang)), th])


def brute_crossing(p, surf_kind, surf_pos, bz, l_min=1e-4, kappa=KAPPA, n_grid=200001):
    """Smallest l > l_min in the first half turn with r(l) = R (kind 0) or
    z(l) = Z (kind 1), by dense sampling then bisection; None if none."""
    w = -kappa * bz * p[3]
    l_max = np.pi / abs(w) if w != 0 else 1e4
    ls = np.linspace(l_min, l_max * (1 - 1e-12), n_grid)

    def g(l):
        s = centre_form(p, l, bz, kappa) if w != 0 else np.array(
            [p[0] + l * np.cos(p[4]), p[1] + l * np.sin(p[4]), p[2] + l / np.tan(p[5])])
        if surf_kind == 0:
            return s[0] ** 2 + s[1] ** 2 - surf_pos ** 2
        return s[2] - surf_pos

    gv = np.array([g(l) for l in ls]) if n_grid < 2000 else _gvec(p, ls, surf_kind, surf_pos, bz, kappa)
    sgn = np.sign(gv)
    ch = np.nonzero(sgn[:-1] * sgn[1:] <= 0)[0]
    if ch.size == 0:
        return None
    a, b = ls[ch[0]], ls[ch[0] + 1]
    ga = g(a)
    for _ in range(200):
        m = 0.5 * (a + b)
        gm = g(m)
        if gm == 0 or b - a < 1e-15 * max(1.0, m):
            a = b = m
            break
        if np.sign(gm) == np.sign(ga):
            a, ga = m, gm
        else:
            b = m
    return 0.5 * (a + b)


def _gvec(p, ls, kind, pos, bz, kappa):
    x, y, z, ipt, phi, th = p
    w = -kappa * bz * ipt
    if w != 0:
        cx, cy = x - np.sin(phi) / w, y + np.cos(phi) / w
        ang = phi + w * ls
        X, Y = cx + np.sin(ang) / w, cy - np.cos(ang) / w
    else:
        X, Y = x + ls * np.cos(phi), y + ls * np.sin(phi)
    Z = z + ls / np.tan(th)
    return X ** 2 + Y ** 2 - pos ** 2 if kind == 0 else Z - pos


def crossing_state(p, kind, pos, bz, kappa=KAPPA):
    """Exact state at the first crossing, by circle geometry (barrel: the
    intersection of the track circle with r = R; disk: linear z).  Returns
    None if there is none within the half turn.  Used as an independent map
    for finite differences."""
    x, y, z, ipt, phi, th = p
    w = -kappa * bz * ipt
    rho = 1.0 / abs(w)
    cx, cy = x - np.sin(phi) / w, y + np.cos(phi) / w
    if kind == 1:
        l = (pos - z) * np.tan(th)
        if not (l > 1e-4 and abs(w) * l < np.pi):
            return None
        return centre_form(p, l, bz, kappa)
    d = np.hypot(cx, cy)
    a = (pos ** 2 - rho ** 2 + d ** 2) / (2 * d)
    hh2 = pos ** 2 - a ** 2
    if hh2 < 0:
        return None
    hh = np.sqrt(hh2)
    best = None
    b0 = np.arctan2(y - cy, x - cx)
    for s in (1, -1):
        px = a * cx / d - s * hh * cy / d
        py = a * cy / d + s * hh * cx / d
        b = np.arctan2(py - cy, px - cx)
        turn = np.mod(np.sign(w) * (b - b0), 2 * np.pi)
        l = turn * rho
        if l > 1e-4 and turn < np.pi and (best is None or l < best):
            best = l
    if best is None:
        return None
    return centre_form(p, best, bz, kappa)
