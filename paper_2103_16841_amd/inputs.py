"""Seeded synthetic inputs: space-time meshes, densities and evaluation points.

This module holds geometry generation only (no quadrature, no kernel, no
part of the method's arithmetic), so that the HIP path and the oracle can be
fed the same arrays.  Meshes follow the paper's workloads: the cube
(-1/2, 1/2)^3 of Sec. 4 and spherical scatterers (Exp. 3), each spatial
triangle extruded over time slabs and split into three tetrahedra; the
lateral boundary Sigma = (0, T) x Gamma is meshed by vertical panels
(Sec. 2, Sec. 3 def. st_be).

Conventions
-----------
* vertex array ``vtx``: float64 [V, 4] = (t, x, y, z);
* tetrahedra ``tets``: int32 [N, 4]; numbered (triangle, slab, sub-tet) so
  that the 3*S panels over one spatial triangle are contiguous;
* prism split for a triangle with global vertex ids i < j < k and slab n:
  {i_n, j_n, k_n, i_n+1}, {j_n, k_n, i_n+1, j_n+1}, {k_n, i_n+1, j_n+1, k_n+1};
  every lateral quad is cut from the larger id at level n to the smaller id
  at level n+1, so neighbouring columns conform;
* jitter: time levels 1..S-1 of every spatial vertex move by an independent
  U(-j dt, j dt); levels 0 and S stay fixed, so the panels stay vertical.
"""
import numpy as np

__all__ = ["cube_surface", "icosphere", "extrude", "cube_mesh", "icosphere_mesh",
           "density_normal", "density_time", "shell_points", "batch_mix", "Mesh"]


class Mesh:
    """A space-time surface mesh (vertices (t,x,y,z), tetrahedra)."""

    def __init__(self, vtx, tets, tri, S, T, name=""):
        self.vtx = np.ascontiguousarray(vtx, dtype=np.float64)
        self.tets = np.ascontiguousarray(tets, dtype=np.int32)
        self.tri = tri
        self.S = S
        self.T = T
        self.name = name

    @property
    def nt(self):
        return int(self.tets.shape[0])

    @property
    def nv(self):
        return int(self.vtx.shape[0])

    def tet_coords(self):
        return self.vtx[self.tets]          # [N, 4, 4]

    def centroid_times(self):
        return self.vtx[self.tets][:, :, 0].mean(axis=1)

    def outward_normals(self):
        """Unit spatial normal of every panel pointing away from the origin
        (the outward normal of Gamma for the cube and the icospheres, which
        are star-shaped about the origin): float64 [N, 3]."""
        X = self.vtx[self.tets][:, :, 1:]            # [N, 4, 3] spatial points
        best = np.zeros((self.nt, 3))
        for a, b, c in ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)):
            v = np.cross(X[:, b] - X[:, a], X[:, c] - X[:, a])
            take = np.einsum("ij,ij->i", v, v) > np.einsum("ij,ij->i", best, best)
            best[take] = v[take]
        n = best / np.linalg.norm(best, axis=1, keepdims=True)
        flip = np.einsum("ij,ij->i", n, X.mean(axis=1)) < 0.0
        n[flip] = -n[flip]
        return n

    def __repr__(self):
        return "Mesh(%s, N=%d, V=%d, S=%d, T=%g)" % (self.name, self.nt, self.nv, self.S, self.T)


def cube_surface():
    """Surface of (-1/2,1/2)^3: 8 vertices, 12 triangles.

    Vertex index = 4[x>0] + 2[y>0] + [z>0]; each face is split along the
    diagonal through its lowest-index vertex.
    """
    pts = np.array([[(i >> 2) & 1, (i >> 1) & 1, i & 1] for i in range(8)], float) - 0.5
    tris = []
    for axis in range(3):
        for side in (0, 1):
            ids = [i for i in range(8) if ((i >> (2 - axis)) & 1) == side]
            lo = min(ids)
            # quad corners in cyclic order around the face
            others = [i for i in ids if i != lo]
            far = max(others, key=lambda m: bin(m ^ lo).count("1"))
            mid = [m for m in others if m != far]
            tris.append(sorted([lo, mid[0], far]))
            tris.append(sorted([lo, mid[1], far]))
    return pts, np.array(tris, dtype=np.int64)


def cube_surface_refined(level):
    """cube_surface() with `level` midpoint subdivisions of every triangle
    (12 * 4^level triangles, vertices on the cube's faces)."""
    pts, tris = cube_surface()
    verts = [p for p in pts]
    faces = [tuple(t) for t in tris]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                verts.append(0.5 * (verts[a] + verts[b]))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.array(verts), np.array([sorted(f) for f in faces], dtype=np.int64)


def icosphere(level):
    """Unit icosphere: icosahedron with `level` midpoint subdivisions."""
    p = (1.0 + 5 ** 0.5) / 2.0
    v = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0), (0, -1, p), (0, 1, p), (0, -1, -p),
         (0, 1, -p), (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    verts = [np.array(x, float) / np.linalg.norm(x) for x in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
             (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
             (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.array(verts), np.array([sorted(f) for f in faces], dtype=np.int64)


def extrude(pts, tris, S, T, jitter=0.0, rng=None, name=""):
    """Triangle surface x [0,T] with S slabs -> vertical tetrahedral panels."""
    nvs = pts.shape[0]
    dt = T / S
    times = np.repeat((np.arange(S + 1) * dt)[:, None], nvs, axis=1)   # [S+1, nvs]
    if jitter > 0.0 and S > 1:
        rng = np.random.default_rng(0) if rng is None else rng
        times[1:S] += rng.uniform(-jitter * dt, jitter * dt, size=(S - 1, nvs))
    vtx = np.zeros(((S + 1) * nvs, 4))
    for n in range(S + 1):
        vtx[n * nvs:(n + 1) * nvs, 0] = times[n]
        vtx[n * nvs:(n + 1) * nvs, 1:] = pts
    tris = np.sort(np.asarray(tris), axis=1)
    ntri = tris.shape[0]
    tets = np.zeros((ntri, S, 3, 4), dtype=np.int64)
    n = np.arange(S)
    for f in range(ntri):
        i, j, k = tris[f]
        I0, J0, K0 = n * nvs + i, n * nvs + j, n * nvs + k
        I1, J1, K1 = I0 + nvs, J0 + nvs, K0 + nvs
        tets[f, :, 0] = np.stack([I0, J0, K0, I1], axis=1)
        tets[f, :, 1] = np.stack([J0, K0, I1, J1], axis=1)
        tets[f, :, 2] = np.stack([K0, I1, J1, K1], axis=1)
    return Mesh(vtx, tets.reshape(-1, 4).astype(np.int32), tris, S, T, name)


def cube_mesh(S=4, T=2.0, jitter=0.0, seed=0, level=0):
    """Unit-cube surface x (0,T), S slabs (144 panels for S=4); level > 0:
    the surface triangles subdivided level times."""
    pts, tris = cube_surface() if level == 0 else cube_surface_refined(level)
    rng = np.random.default_rng(seed)
    name = "cube_S%d_T%g" % (S, T) if level == 0 else "cube_L%d_S%d_T%g" % (level, S, T)
    return extrude(pts, tris, S, T, jitter, rng, name=name)


def icosphere_mesh(level=2, S=32, T=4.0, jitter=0.2, seed=2):
    """Icosphere of radius 1 x (0,T), S slabs, jittered interior levels."""
    pts, tris = icosphere(level)
    rng = np.random.default_rng(seed)
    return extrude(pts, tris, S, T, jitter, rng,
                   name="icosphere_L%d_S%d_T%g_j%g" % (level, S, T, jitter))


def density_normal(n, seed=0):
    return np.random.default_rng(seed).standard_normal(n)


def density_time(mesh, f):
    """w_j = f(t of panel j's centroid)."""
    return np.asarray(f(mesh.centroid_times()), dtype=np.float64)


def shell_points(n, T, rmin=1.5, rmax=3.0, seed=0):
    """Points (t,x,y,z): uniform direction, |x| uniform in volume on the
    shell [rmin, rmax], t ~ U[0, T]."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    u = rng.uniform(size=n)
    r = (rmin ** 3 + u * (rmax ** 3 - rmin ** 3)) ** (1.0 / 3.0)
    t = rng.uniform(0.0, T, size=n)
    return np.concatenate([t[:, None], d * r[:, None]], axis=1)


def batch_mix(count=64, seed=3, T=4.0, jitter=0.2, levels=(0, 4), slabs=(8, 65)):
    """Mix of icosphere meshes: level ~ U{0..3}, S ~ U{8..64}, then jitter."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        L = int(rng.integers(*levels))
        S = int(rng.integers(*slabs))
        pts, tris = icosphere(L)
        out.append(extrude(pts, tris, S, T, jitter, rng,
                           name="icosphere_L%d_S%d_T%g_j%g" % (L, S, T, jitter)))
    return out
