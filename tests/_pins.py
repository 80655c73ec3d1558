"""Independent reference computations used to pin the oracle.

Nothing here shares code with the oracle or the HIP path: closed forms are
written from their textbook / paper statements, brute force uses bisection
and adaptive quadrature with no root formulas and no breakpoint logic.
"""
import math

import mpmath as mp
import numpy as np
from scipy import integrate


# --- appendix closed forms (apex in the panel plane, large panel) --------
# The tet is conv{h e1, h e2, h e3, 0} in (tau, y1, y2, y3) with normal e4;
# k = 1/|x-y| without the 4 pi.  Case 2 (edge) as printed; Case 1 (corner)
# with the printed eps^2/(4 t^2) under the root replaced by eps^2/(2 t^2).

def appendix_case2(t, e):
    t, e = mp.mpf(t), mp.mpf(e)
    return 2 * t * (mp.pi - mp.acos(-e / t)) - 2 * e * mp.log((1 + mp.sqrt(1 - e * e / (t * t))) / (e / t))


def appendix_case1(t, e, printed=False):
    t, e = mp.mpf(t), mp.mpf(e)
    s2 = mp.sqrt(2)
    q = 4 if printed else 2
    return (2 * t * (mp.pi / 4 - mp.asin(s2 / 2 * e / t)) - s2 * e * mp.log(s2 - 1)
            + s2 * e * mp.log(s2 * (1 - mp.sqrt(1 - e * e / (q * t * t))) / (e / t)))


def appendix_tet(h=50.0):
    # rows (t, x, y, z)
    return np.array([[h, 0, 0, 0], [0, h, 0, 0], [0, 0, h, 0], [0, 0, 0, 0]], float)


# --- Laplace single layer of a flat triangle (Wilton et al. type formula) --

def triangle_laplace(x, tri):
    """int_T dA(y) / |x - y| for a flat triangle tri (3x3) and point x."""
    tri = np.asarray(tri, float)
    x = np.asarray(x, float)
    n = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    n /= np.linalg.norm(n)
    d = float(np.dot(x - tri[0], n))
    p = x - d * n
    ad = abs(d)
    total = 0.0
    for i in range(3):
        a, b = tri[i], tri[(i + 1) % 3]
        L = np.linalg.norm(b - a)
        s_hat = (b - a) / L
        m = np.cross(s_hat, n)                   # outward edge normal (ccw w.r.t. n)
        t0 = float(np.dot(a - p, m))             # signed distance of p to edge line
        sm = float(np.dot(a - p, s_hat))
        sp = float(np.dot(b - p, s_hat))
        R0sq = t0 * t0 + d * d
        Rm = math.sqrt(sm * sm + R0sq)
        Rp = math.sqrt(sp * sp + R0sq)
        if abs(t0) > 0.0:
            # log term; written with the stable ratio form
            if sp + Rp > 0 and sm + Rm > 0:
                lg = math.log((Rp + sp) / (Rm + sm))
            else:
                lg = math.log((Rm - sm) / (Rp - sp))
            total += t0 * lg
        if ad > 0.0:
            total -= ad * (math.atan2(t0 * sp, R0sq + ad * Rp) - math.atan2(t0 * sm, R0sq + ad * Rm))
    return total


def triangle_laplace_quad(x, tri):
    """Same integral by adaptive 2-D quadrature (Duffy-free, for checking)."""
    tri = np.asarray(tri, float)
    x = np.asarray(x, float)
    A, B, C = tri
    J = np.linalg.norm(np.cross(B - A, C - A))

    def f(v, u):
        y = A + u * (B - A) + v * (C - A)
        return 1.0 / np.linalg.norm(x - y)

    val, _ = integrate.dblquad(f, 0, 1, 0, lambda u: 1 - u, epsabs=1e-13, epsrel=1e-12)
    return val * J


# --- ray / triangle clipping in the panel plane -----------------------------

def _ray_interval(p, e, tri2):
    """Interval {s >= 0 : p + s e in triangle} for a 2-D triangle (3x2)."""
    lo, hi = 0.0, math.inf
    cen = tri2.mean(axis=0)
    for i in range(3):
        a, b = tri2[i], tri2[(i + 1) % 3]
        m = np.array([b[1] - a[1], a[0] - b[0]])
        if np.dot(cen - a, m) < 0:
            m = -m                               # inward normal
        num = -float(np.dot(p - a, m))           # need s * (e.m) >= num
        den = float(np.dot(e, m))
        if den == 0.0:
            if num > 0:
                return None
        elif den > 0:
            lo = max(lo, num / den)
        else:
            hi = min(hi, num / den)
    if hi <= lo:
        return None
    return lo, hi


def triangle_ball_potential(x, tri, R):
    """int_{T cap {|x-y| < R}} dA / |x - y| by 1-D adaptive quadrature in the
    polar angle about the foot point: with s the in-plane radius and
    r = sqrt(s^2 + d^2) one has dA/|x-y| = dr dphi, so the inner integral is
    min(r(s2), R) - min(r(s1), R)."""
    tri = np.asarray(tri, float)
    x = np.asarray(x, float)
    n = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    n /= np.linalg.norm(n)
    e1 = (tri[1] - tri[0]) / np.linalg.norm(tri[1] - tri[0])
    e2 = np.cross(n, e1)
    d = float(np.dot(x - tri[0], n))
    p3 = x - d * n
    tri2 = np.array([[np.dot(v - p3, e1), np.dot(v - p3, e2)] for v in tri])
    p = np.zeros(2)

    def F(s):
        return min(math.sqrt(s * s + d * d), R)

    def g(phi):
        iv = _ray_interval(p, np.array([math.cos(phi), math.sin(phi)]), tri2)
        if iv is None:
            return 0.0
        return max(F(iv[1]) - F(iv[0]), 0.0)

    pts = sorted(math.atan2(v[1], v[0]) % (2 * math.pi) for v in tri2)
    edges = [0.0] + pts + [2 * math.pi]
    tot = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        if b > a:
            val, _ = integrate.quad(g, a, b, limit=400, epsabs=1e-14, epsrel=1e-13)
            tot += val
    return tot


# --- brute force L(phi) and inner integral ---------------------------------

def _face_halfspaces_4d(tet):
    """Half-spaces of the panel in (t, y) coordinates of its own hyperplane,
    built from scratch: returns (frame, list of (normal3, offset))."""
    tet = np.asarray(tet, float)
    X = tet[:, 1:]
    # plane of the spatial projection by SVD (independent of the oracle's frame)
    c = X.mean(axis=0)
    _, _, vt = np.linalg.svd(X - c)
    n = vt[2]
    e1, e2 = vt[0], vt[1]
    V = np.array([[v[0], np.dot(v[1:] - c, e1), np.dot(v[1:] - c, e2)] for v in tet])
    faces = []
    for k in range(4):
        idx = [m for m in range(4) if m != k]
        N = np.cross(V[idx[1]] - V[idx[0]], V[idx[2]] - V[idx[0]])
        if np.dot(N, V[k] - V[idx[0]]) > 0:
            N = -N
        faces.append((N, float(np.dot(N, V[idx[0]]))))
    return (c, e1, e2, n), V, faces


def brute_L(x4, tet, phi, ngrid=4000, frame=None):
    """L(phi) by grid search + bisection of the face level function along r
    (no root formulas): measure of {r >= |d|: point inside the open tet}.
    phi is measured from frame[0] towards frame[1] (two orthonormal vectors
    spanning the panel plane); default: this module's own frame."""
    (c, e1, e2, n), V, faces = _face_halfspaces_4d(tet)
    if frame is not None:
        f1, f2 = np.asarray(frame[0], float), np.asarray(frame[1], float)
        dv = math.cos(phi) * f1 + math.sin(phi) * f2
        phi = math.atan2(float(np.dot(dv, e2)), float(np.dot(dv, e1)))
    t = x4[0]
    xv = np.asarray(x4[1:]) - c
    pu, pv, d = float(np.dot(xv, e1)), float(np.dot(xv, e2)), float(np.dot(xv, n))
    rlo, rhi = abs(d), t - V[:, 0].min()
    if rhi <= rlo:
        return 0.0
    cs, sn = math.cos(phi), math.sin(phi)

    def level(r):
        s = math.sqrt(max(r * r - d * d, 0.0))
        P = np.array([t - r, pu + s * cs, pv + s * sn])
        return max(float(np.dot(N, P) - h) for N, h in faces)

    rs = np.linspace(rlo, rhi, ngrid)
    ss = np.sqrt(np.maximum(rs * rs - d * d, 0.0))
    Pg = np.stack([t - rs, pu + ss * cs, pv + ss * sn], axis=1)
    Nm = np.array([N for N, _ in faces])
    hm = np.array([h for _, h in faces])
    vals = (Pg @ Nm.T - hm).max(axis=1)
    inside = vals < 0
    # thin admissible pieces between grid points: golden-section search of
    # the level function around every positive local minimum
    gr = (math.sqrt(5) - 1) / 2
    extra = 0.0
    for i in range(1, ngrid - 1):
        if inside[i] or not (vals[i] <= vals[i - 1] and vals[i] <= vals[i + 1]):
            continue
        a, b = rs[i - 1], rs[i + 1]
        c1, c2 = b - gr * (b - a), a + gr * (b - a)
        f1, f2 = level(c1), level(c2)
        for _ in range(100):
            if f1 < f2:
                b, c2, f2 = c2, c1, f1
                c1 = b - gr * (b - a)
                f1 = level(c1)
            else:
                a, c1, f1 = c1, c2, f2
                c2 = a + gr * (b - a)
                f2 = level(c2)
        rm = 0.5 * (a + b)
        if level(rm) < 0:
            def bis_out(lo_in, hi_out):
                for _ in range(100):
                    m = 0.5 * (lo_in + hi_out)
                    if level(m) < 0:
                        lo_in = m
                    else:
                        hi_out = m
                return 0.5 * (lo_in + hi_out)
            extra += bis_out(rm, rs[i + 1]) - bis_out(rm, rs[i - 1])
    tot = extra
    i = 0
    while i < ngrid:
        if not inside[i]:
            i += 1
            continue
        j = i
        while j + 1 < ngrid and inside[j + 1]:
            j += 1
        # refine both ends by bisection
        def bis(a, b, want_inside_at_b):
            for _ in range(80):
                m = 0.5 * (a + b)
                if (level(m) < 0) == want_inside_at_b:
                    b = m
                else:
                    a = m
            return 0.5 * (a + b)
        left = rs[i] if i == 0 else bis(rs[i - 1], rs[i], True)
        right = rs[j] if j == ngrid - 1 else bis(rs[j + 1], rs[j], True)
        tot += right - left
        i = j + 1
    return tot


def brute_inner(x4, tet, ngrid=20000, pieces=64):
    """(1/4pi) int L dphi by adaptive Gauss-Kronrod quadrature of brute_L
    on equal pieces of [0, 2pi] (no breakpoint information)."""
    f = lambda ph: brute_L(x4, tet, float(ph), ngrid)
    cuts = np.linspace(0, 2 * math.pi, pieces + 1)
    tot = 0.0
    for a, b in zip(cuts[:-1], cuts[1:]):
        val, _ = integrate.quad(f, a, b, limit=100, epsabs=1e-11, epsrel=1e-10)
        tot += val
    return tot / (4 * math.pi)


# --- misc geometry -----------------------------------------------------------

def tet_volume3(tet):
    """3-volume of a vertical panel inside its hyperplane (R x plane)."""
    (c, e1, e2, n), V, _ = _face_halfspaces_4d(tet)
    return abs(np.linalg.det(np.array([V[1] - V[0], V[2] - V[0], V[3] - V[0]]))) / 6.0


def random_rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q *= np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


# --- a wave from a point source (Kirchhoff's formula checks) ---------------

POINT_SOURCE = np.array([0.0, 0.0, 2.5])


def _pulse(t):
    """sin^2(pi t / 2) on (0, 2), zero outside (C^1)."""
    return np.where((t > 0.0) & (t < 2.0), np.sin(0.5 * np.pi * t) ** 2, 0.0)


def _pulse_dt(t):
    return np.where((t > 0.0) & (t < 2.0), 0.5 * np.pi * np.sin(np.pi * t), 0.0)


def point_source_wave(p):
    """u(t, x) = f(t - |x - x0|) / (4 pi |x - x0|) with x0 = (0, 0, 2.5): a
    solution of the wave equation away from x0 (inside the unit sphere),
    zero at times t <= |x - x0|.  p: [..., 4] points (t, x, y, z)."""
    r = np.linalg.norm(p[..., 1:] - POINT_SOURCE, axis=-1)
    return _pulse(p[..., 0] - r) / (4.0 * np.pi * r)


def point_source_wave_dn(p, n):
    """Normal derivative <grad_x u, n> of point_source_wave at points p."""
    y = p[..., 1:]
    r = np.linalg.norm(y - POINT_SOURCE, axis=-1)
    tr = p[..., 0] - r
    g = (-_pulse_dt(tr) / (4.0 * np.pi * r) - _pulse(tr) / (4.0 * np.pi * r * r))[..., None] \
        * (y - POINT_SOURCE) / r[..., None]
    return np.einsum("...i,...i->...", g, n)


# --- a panel whose cone sections have no breakpoints ---------------------

BIG_TET = np.array([[0.0, -10.0, -10.0, 0.0], [0.0, 10.0, -10.0, 0.0], [0.0, 0.0, 10.0, 0.0],
                    [20.0, 0.0, 0.0, 0.0]])
BIG_TET_POINTS = [[2.0, 0.0, 0.0, 0.5], [3.0, 0.5, -0.3, 0.8], [1.5, 1.0, 1.0, -0.3]]


def big_tet_closed_form(x4, vv, sgn=1.0):
    """No breakpoints: the whole cone section r in [|d|, t - tmin] lies in
    the panel, so the gamma term integrates to 0 over the circle and
    D v = (d_n / 2) v(t, p) (1/|d| - 1/(t - tmin))."""
    t, x, y, z = x4
    M = np.column_stack([np.ones(4), BIG_TET[:, :3]])          # v = c0 + c_t t + c_x x + c_y y
    c = np.linalg.solve(M, np.asarray(vv, float))
    alpha = c[0] + c[1] * t + c[2] * x + c[3] * y
    dn = sgn * z
    return 0.5 * dn * alpha * (1.0 / abs(z) - 1.0 / (t - BIG_TET[:, 0].min()))
