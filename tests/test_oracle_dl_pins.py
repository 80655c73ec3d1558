"""Pins of the oracle's retarded double-layer potential (eq. dlp with the
kernels k2, k3 of eq. kfunc) against what the mathematics fixes:

* static columns (every retarded time inside the column's time range): a
  constant density gives the solid angle of the triangle (closed form of
  Van Oosterom and Strackee), v = tau gives t times it (the k2 term), and a
  spatially linear density gives the 2-D integral of k3 v over the triangle
  (adaptive quadrature of the definition);
* Gauss's law on closed polyhedral surfaces: D 1 = -1 inside, 0 outside;
* truncated columns (the light cone leaves the time range inside the
  triangle): the definition k3 v(t - r, y) + k2 dv/dtau integrated by
  nested adaptive quadrature in polar coordinates about the foot point;
* additivity: a column split in time gives the same sum;
* on the surface (direct value): K 1 = -1/2 at points inside the faces of
  a closed polyhedral surface, hence the energetic form b_K(tau, phi_i) =
  -1/2 sum_q w_iq t_q; b_I of an affine function is its outer-rule sum;
* Kirchhoff's formula: inside the sphere a wave from an outside point
  source equals S(du/dn) - D(u) of its traces, to the discretisation error,
  which falls under refinement (with the single layer's oracle).
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from paper_2103_16841_amd import inputs
from _pins import (_ray_interval, point_source_wave, point_source_wave_dn, BIG_TET,
                   BIG_TET_POINTS, big_tet_closed_form)

FOUR_PI = 4.0 * math.pi


def column(tri, ta, tb):
    """Three tetrahedra filling [ta, tb] x triangle (the extrusion split)."""
    tri = np.asarray(tri, float)
    lo = [np.array([ta, *p]) for p in tri]
    hi = [np.array([tb, *p]) for p in tri]
    return [np.array([lo[0], lo[1], lo[2], hi[0]]), np.array([lo[1], lo[2], hi[0], hi[1]]),
            np.array([lo[2], hi[0], hi[1], hi[2]])]


def tri_normal(tri):
    n = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    return n / np.linalg.norm(n)


def solid_angle(x, tri):
    """Omega_n(x) = int_T <n, y - x> / |y - x|^3 dA for n = the normal of the
    vertex order (Van Oosterom and Strackee)."""
    R = [np.asarray(p, float) - x for p in tri]
    l = [np.linalg.norm(r) for r in R]
    num = np.dot(R[0], np.cross(R[1], R[2]))
    den = l[0] * l[1] * l[2] + np.dot(R[0], R[1]) * l[2] + np.dot(R[0], R[2]) * l[1] \
        + np.dot(R[1], R[2]) * l[0]
    return 2.0 * math.atan2(num, den)


def dl_column(x4, tets, n, vfun, n_g=32):
    return sum(oracle.inner_dl(x4, T, n, [vfun(p) for p in T], n_g=n_g) for T in tets)


# The phi-rule's own error: with the default 16 nodes per piece it reaches
# about 1e-7 where the foot point lies near a panel edge (the single layer's
# rule converges alike there); it falls to rounding level by 32-96 nodes.
# The exact identities are checked with 32 (one column) or 64 nodes (closed
# surfaces), the default rule at 2e-7.


TRI = np.array([[0.1, -0.2, 0.05], [0.9, 0.1, -0.1], [0.2, 0.7, 0.3]])


@pytest.mark.parametrize("x", [(0.3, 0.2, 0.6), (0.4, 0.1, -0.5), (1.2, 0.9, 0.2),
                               (0.35, 0.2, 0.13), (-0.6, -0.4, -0.3)])
def test_static_solid_angle_and_time_linear(x):
    x = np.array(x)
    n = tri_normal(TRI)
    r = [np.linalg.norm(p - x) for p in TRI]
    t = max(r) + 1.0           # every retarded time t - |x - y| in (0, 3)
    tets = column(TRI, 0.0, 3.0)
    om = solid_angle(x, TRI)
    x4 = np.array([t, *x])
    d1 = dl_column(x4, tets, n, lambda p: 1.0)
    assert abs(d1 - (-om / FOUR_PI)) <= 1e-11 * max(1.0, abs(om))
    # v = tau: k3 (t - r) / ... + k2 * 1 = t k3 (static), the k2 term at work
    dt = dl_column(x4, tets, n, lambda p: p[0])
    assert abs(dt - (-t * om / FOUR_PI)) <= 1e-11 * t
    # the outward normal's sign flips the potential
    assert abs(dl_column(x4, tets, -n, lambda p: 1.0) + d1) <= 1e-15
    d16 = dl_column(x4, tets, n, lambda p: 1.0, n_g=oracle.DEFAULT_NG)
    assert abs(d16 - (-om / FOUR_PI)) <= 2e-7 * max(1.0, abs(om))


def _static_linear_brute(x, tri, n, a, c0):
    A, B, C = tri
    J = np.linalg.norm(np.cross(B - A, C - A))

    def f(v, u):
        y = A + u * (B - A) + v * (C - A)
        d = x - y
        r = np.linalg.norm(d)
        return np.dot(n, d) * (c0 + np.dot(a, y)) / (FOUR_PI * r ** 3)

    val, _ = integrate.dblquad(f, 0, 1, 0, lambda u: 1 - u, epsabs=1e-14, epsrel=1e-12)
    return val * J


@pytest.mark.parametrize("x", [(0.3, 0.2, 0.6), (1.1, 0.8, -0.4), (0.2, 0.1, 0.5)])
def test_static_spatially_linear(x):
    x = np.array(x)
    n = tri_normal(TRI)
    a = np.array([0.7, -1.3, 0.4])
    c0 = 0.25
    t = max(np.linalg.norm(p - x) for p in TRI) + 1.0
    got = dl_column(np.array([t, *x]), column(TRI, 0.0, 3.0), n, lambda p: c0 + np.dot(a, p[1:]))
    ref = _static_linear_brute(x, TRI, n, a, c0)
    assert abs(got - ref) <= 1e-10 * max(1.0, abs(ref))


def _truncated_brute(x4, tri, n, ta, tb, vfun, dvdtau):
    """int over {y in T : ta < t - |x - y| < tb} of k3 v(t - r, y) + k2 dv/dtau
    (eq. dlp after the delta), by nested adaptive quadrature in polar
    coordinates (s, phi) about the foot point p of x on the plane."""
    t, x = x4[0], np.asarray(x4[1:], float)
    e1 = (tri[1] - tri[0]) / np.linalg.norm(tri[1] - tri[0])
    e2 = np.cross(n, e1)
    d = float(np.dot(x - tri[0], n))
    p3 = x - d * n
    tri2 = np.array([[np.dot(v - p3, e1), np.dot(v - p3, e2)] for v in tri])
    rlo, rhi = max(abs(d), t - tb), t - ta
    slo = math.sqrt(max(rlo * rlo - d * d, 0.0))
    shi = math.sqrt(max(rhi * rhi - d * d, 0.0))

    def inner(phi):
        e = np.array([math.cos(phi), math.sin(phi)])
        iv = _ray_interval(np.zeros(2), e, tri2)
        if iv is None:
            return 0.0
        s0, s1 = max(iv[0], slo), min(iv[1], shi)
        if not s1 > s0:
            return 0.0
        ev = e[0] * e1 + e[1] * e2

        def f(s):
            y = p3 + s * ev
            r = math.sqrt(s * s + d * d)
            k3 = d / (FOUR_PI * r ** 3)
            k2 = d / (FOUR_PI * r ** 2)
            return (k3 * vfun(t - r, y) + k2 * dvdtau) * s

        val, _ = integrate.quad(f, s0, s1, epsabs=1e-14, epsrel=1e-13, limit=200)
        return val

    cuts = sorted(math.atan2(v[1], v[0]) % (2 * math.pi) for v in tri2)
    edges = [0.0] + cuts + [2 * math.pi]
    tot = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        if hi > lo:
            val, _ = integrate.quad(inner, lo, hi, limit=400, epsabs=1e-13, epsrel=1e-12)
            tot += val
    return tot


@pytest.mark.parametrize("x,t", [((0.3, 0.2, 0.6), 1.2), ((0.5, 0.3, -0.25), 0.9),
                                 ((1.0, 0.6, 0.3), 1.4)])
def test_truncated_column_against_definition(x, t):
    x = np.array(x)
    n = tri_normal(TRI)
    ta, tb = 0.0, 0.6
    x4 = np.array([t, *x])
    tets = column(TRI, ta, tb)
    r = [np.linalg.norm(p - x) for p in TRI]
    assert min(r) < t - ta or max(r) > t - tb     # the cone cuts the column
    a = np.array([0.3, 0.8, -0.5])
    got = dl_column(x4, tets, n, lambda p: 0.4 + 1.5 * p[0] + np.dot(a, p[1:]))
    ref = _truncated_brute(x4, TRI, n, ta, tb, lambda tau, y: 0.4 + 1.5 * tau + np.dot(a, y), 1.5)
    assert abs(ref) > 1e-3
    assert abs(got - ref) <= 1e-9 * max(1.0, abs(ref))


def test_time_split_additivity():
    x4 = np.array([1.3, 0.35, 0.25, 0.4])
    n = tri_normal(TRI)
    v = lambda p: 1.0 - 0.7 * p[0] + 0.4 * p[1] - 0.9 * p[3]
    whole = dl_column(x4, column(TRI, 0.0, 1.0), n, v)
    split = dl_column(x4, column(TRI, 0.0, 0.37), n, v) + dl_column(x4, column(TRI, 0.37, 1.0), n, v)
    assert abs(whole) > 1e-3
    assert abs(whole - split) <= 1e-12 * max(1.0, abs(whole))


@pytest.mark.parametrize("level,S,jitter", [(1, 1, 0.0), (1, 3, 0.2), (2, 2, 0.2)])
def test_gauss_closed_surface(level, S, jitter):
    mesh = inputs.icosphere_mesh(level=level, S=S, T=6.0, jitter=jitter, seed=4)
    nrm = mesh.outward_normals()
    ones = np.ones(mesh.nv)
    inside = np.array([[5.0, 0.0, 0.0, 0.0], [5.0, 0.3, -0.2, 0.4], [4.8, -0.5, 0.1, 0.2]])
    outside = np.array([[5.0, 1.6, 0.0, 0.3], [5.5, -0.9, 1.3, -0.8]])
    for n_g, tol in ((64, 1e-10), (oracle.DEFAULT_NG, 2e-7)):
        u_in = oracle.potential_dl(mesh.vtx, mesh.tets, nrm, ones, inside, n_g=n_g)
        u_out = oracle.potential_dl(mesh.vtx, mesh.tets, nrm, ones, outside, n_g=n_g)
        assert np.all(np.abs(u_in + 1.0) <= tol)
        assert np.all(np.abs(u_out) <= tol)


def test_in_plane_and_argument_errors():
    tets = column(TRI, 0.0, 3.0)
    n = tri_normal(TRI)
    x_in = 0.3 * TRI[0] + 0.3 * TRI[1] + 0.4 * TRI[2]
    assert oracle.inner_dl([1.0, *x_in], tets[0], n, [1, 2, 3, 4]) == 0.0
    with pytest.raises(ValueError):
        oracle.inner_dl([1.0, 0.3, 0.2, 0.6], tets[0], np.cross(n, TRI[1] - TRI[0]), [1, 1, 1, 1])


def test_kirchhoff_representation():
    """u = S(du/dn) - D(u) inside (interior problem, outward normal; D 1 = -1
    inside fixes the sign): D of the vertex interpolant of u (V_h^1), S of
    du/dn at the panel centroids (S_h^0).  A wrong sign of the k2 term
    would leave an O(1) error."""
    pts = np.array([[3.5, 0.0, 0.0, 0.3], [3.2, 0.2, -0.3, 0.0], [3.8, -0.2, 0.1, -0.4]])
    exact = point_source_wave(pts)
    errs = []
    for level, S in ((2, 16), (3, 32)):
        mesh = inputs.icosphere_mesh(level=level, S=S, T=4.0, jitter=0.0, seed=0)
        nrm = mesh.outward_normals()
        cen = mesh.vtx[mesh.tets].mean(axis=1)
        rep = oracle.potential(mesh.vtx, mesh.tets, point_source_wave_dn(cen, nrm), pts) \
            - oracle.potential_dl(mesh.vtx, mesh.tets, nrm, point_source_wave(mesh.vtx), pts)
        errs.append(np.abs(rep - exact).max() / np.abs(exact).max())
    assert errs[1] < 0.01 and errs[1] < 0.3 * errs[0]


def _static_rows(mesh, k=10):
    """Rows whose outer points see the whole unit sphere inside (0, T)."""
    ct = mesh.centroid_times()
    return np.where((ct > 3.0) & (ct < mesh.T - 0.5))[0][::7][:k]


def test_surface_direct_value_and_energetic_forms():
    mesh = inputs.icosphere_mesh(level=1, S=3, T=6.0, jitter=0.2, seed=4)
    nrm = mesh.outward_normals()
    rows = _static_rows(mesh)
    assert len(rows) >= 5
    P0, _ = oracle.outer_points(mesh.vtx[mesh.tets[rows[0]]])
    # K 1 = -1/2 inside the faces of a closed polyhedron (static)
    k1 = oracle.potential_dl(mesh.vtx, mesh.tets, nrm, np.ones(mesh.nv), P0, n_g=64)
    assert np.all(np.abs(k1 + 0.5) <= 1e-13)
    k16 = oracle.potential_dl(mesh.vtx, mesh.tets, nrm, np.ones(mesh.nv), P0)
    assert np.all(np.abs(k16 + 0.5) <= 2e-7)
    # b_K(tau) = -1/2 sum_q w_q t_q (the k2 term with K 1 = -1/2)
    tv = mesh.vtx[:, 0].copy()
    bk = oracle.dl_energetic_rows(mesh.vtx, mesh.tets, nrm, tv, rows, c_id=0.0, n_g=64)
    ex = np.array([-0.5 * np.dot(W, P[:, 0]) for P, W in
                   (oracle.outer_points(mesh.vtx[mesh.tets[i]]) for i in rows)])
    assert np.all(np.abs(bk - ex) <= 1e-13)
    # b_I of an affine function of (t, x, y, z): its outer-rule sum
    a = np.array([0.3, -0.7, 0.4, 1.1])
    va = 0.2 + mesh.vtx @ a
    bi = oracle.dl_energetic_rows(mesh.vtx, mesh.tets, nrm, va, rows, c_id=1.0) \
        - oracle.dl_energetic_rows(mesh.vtx, mesh.tets, nrm, va, rows, c_id=0.0)
    exi = np.array([np.dot(W, 0.2 + P @ a) for P, W in
                    (oracle.outer_points(mesh.vtx[mesh.tets[i]]) for i in rows)])
    assert np.all(np.abs(bi - exi) <= 1e-14)


# --- the L2 projection onto V_h^1 (eq. df_dir's Q_h^1) -----------------------

def _rule_values(mesh, f):
    P = np.array([oracle.l2_points(mesh.vtx[mesh.tets[j]])[0] for j in range(mesh.nt)])
    return P, f(P)


def test_projection_reproduces_V1():
    """Q_h^1 is a projection: a function of V_h^1 (random vertex values,
    linear on every panel) comes back unchanged."""
    mesh = inputs.icosphere_mesh(level=1, S=3, T=3.0, jitter=0.2, seed=7)
    v = np.random.default_rng(3).standard_normal(mesh.nv)
    # g at the rule points: the panel's linear interpolant of v
    g = np.zeros((mesh.nt, 27))
    for j in range(mesh.nt):
        T = mesh.vtx[mesh.tets[j]]
        P, _ = oracle.l2_points(T)
        # barycentric coordinates of each point in (t, x, y, z): least squares on the panel's affine hull
        E = (T[1:] - T[0]).T                            # 4 x 3
        bc = np.linalg.lstsq(E, (P - T[0]).T, rcond=None)[0].T
        lamq = np.concatenate([1.0 - bc.sum(axis=1, keepdims=True), bc], axis=1)
        g[j] = lamq @ v[mesh.tets[j]]
    c = oracle.l2_projection(mesh.vtx, mesh.tets, g)
    assert np.abs(c - v).max() <= 1e-11


def _tet_volume4(T):
    E = (T[1:] - T[0])
    return math.sqrt(np.linalg.det(E @ E.T)) / 6.0


def test_projection_keeps_integrals_of_quadratics():
    """1 is in V_h^1, so int Q g = int g; for quadratic g the panel integrals
    follow from the 10-point rule (vertices and edge midpoints) exactly."""
    mesh = inputs.icosphere_mesh(level=1, S=3, T=3.0, jitter=0.2, seed=7)
    for f in (lambda p: p[..., 0] ** 2, lambda p: p[..., 1] * p[..., 2] + p[..., 0] * p[..., 3]):
        _, g = _rule_values(mesh, f)
        c = oracle.l2_projection(mesh.vtx, mesh.tets, g)
        iq = ig = 0.0
        for j in range(mesh.nt):
            T = mesh.vtx[mesh.tets[j]]
            vol = _tet_volume4(T)
            iq += vol / 4.0 * c[mesh.tets[j]].sum()
            mids = [0.5 * (T[a] + T[b]) for a in range(4) for b in range(a + 1, 4)]
            ig += vol * (-sum(f(T[a]) for a in range(4)) / 20.0 + sum(f(m) for m in mids) / 5.0)
        assert abs(iq - ig) <= 1e-12 * max(1.0, abs(ig))


@pytest.mark.parametrize("x4", BIG_TET_POINTS)
def test_periodic_case_closed_form(x4):
    assert oracle.breakpoints(x4, BIG_TET).size == 0
    vv = [1.0, 2.0, 3.0, 4.0]
    for sgn in (1.0, -1.0):
        got = oracle.inner_dl(x4, BIG_TET, [0.0, 0.0, sgn], vv)
        assert abs(got - big_tet_closed_form(x4, vv, sgn)) <= 1e-13


def test_cone_through_a_vertex_breaks_there():
    """A point on the light cone of a panel vertex: the cone meets the three
    edges at that vertex, so the vertex's direction is a breakpoint (edge
    events on the closed edges; the roots sit at 0 or 1 only up to
    rounding)."""
    mesh = inputs.icosphere_mesh(level=2, S=16, T=4.0, jitter=0.0, seed=0)
    T = mesh.vtx[mesh.tets[3718]]
    x4 = np.array([4.0, 0.2, -1.6, 0.0])
    k = 2                                           # |x - y_2| = t - tau_2 = 2
    assert abs(np.linalg.norm(x4[1:] - T[k, 1:]) - (x4[0] - T[k, 0])) <= 1e-15
    o, e1, e2, n = oracle.panel_frame(T)
    w = T[k, 1:] - x4[1:]
    ang = math.atan2(w @ e2, w @ e1) % (2.0 * math.pi)
    bp = oracle.breakpoints(x4, T)
    assert np.min(np.abs(bp - ang)) <= 1e-12
