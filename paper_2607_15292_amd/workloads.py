"""Seeded synthetic inputs: boundary meshes, gCQ contour points and right-hand sides.

This module holds input generators only.  It computes no kernel entry, quadrature,
compression or product of the boundary element method, so that the product path and
the independent oracle can both be fed from it without sharing any of the method's
arithmetic.

Meshes are flat-triangle surfaces (the boundary approximation of Sec. 2.3, eq. (tri)).
Triangles are oriented so that (v1 - v0) x (v2 - v0) points out of the bounded body.

* ``cube_grid(n, half)``   -- cube [-half, half]^3, n x n squares per face, each square
  split along its (0,0)-(1,1) diagonal.  n = 4, half = 1 gives 192 triangles / 98 nodes.
* ``paper_cube(level)``    -- the unit-cube family of Table 1 (Sec. 4.1): 2 x 2 squares per
  face, every square cut into 4 triangles about its centre (50 nodes / 96 elements), then
  uniform red refinement (194/384, 770/1536, 3074/6144).
* ``icosphere(level, radius)`` -- icosahedron with midpoint subdivision projected to the
  sphere: 20 * 4**level triangles (1280, 5120, 20480 for levels 3, 4, 5).
* ``pulsating_sphere(points, normals, s)`` -- Dirichlet data and exact traction of the
  radially pulsating unit sphere (exterior domain), the closed-form test problem of the
  solve.
* ``bdf2_contour(L, dt)`` -- the L contour points s_l = (3 - 4 z + z^2) / (2 dt),
  z = R exp(2 pi i l / L), R = (1e-10)**(1 / (2 L)); they come in conjugate pairs
  (Sec. 4.1 notes this property of the gCQ points).
* ``random_rhs(seed, shape)`` -- complex128 a + i b, a, b ~ N(0, 1) i.i.d.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "cube_grid",
    "paper_cube",
    "icosphere",
    "bdf2_contour",
    "random_rhs",
    "mesh_summary",
]


class _NodeTable:
    """Deduplicates nodes by an exact integer key."""

    def __init__(self):
        self.key_to_id = {}
        self.coords = []

    def get(self, key, xyz):
        nid = self.key_to_id.get(key)
        if nid is None:
            nid = len(self.coords)
            self.key_to_id[key] = nid
            self.coords.append(xyz)
        return nid


# (normal axis, sign, u axis, v axis) with u x v = outward normal.
_CUBE_FACES = (
    (0, -1, 2, 1),  # -x : e_z x e_y = -e_x
    (0, +1, 1, 2),  # +x : e_y x e_z = +e_x
    (1, -1, 0, 2),  # -y : e_x x e_z = -e_y
    (1, +1, 2, 0),  # +y : e_z x e_x = +e_y
    (2, -1, 1, 0),  # -z : e_y x e_x = -e_z
    (2, +1, 0, 1),  # +z : e_x x e_y = +e_z
)


def cube_grid(n: int = 4, half: float = 1.0):
    """Cube [-half, half]^3 with n x n squares per face, 2 triangles per square.

    Faces come in the order -x, +x, -y, +y, -z, +z; squares in (u, v) row-major order;
    each square (p00, p10, p11, p01) gives triangles (p00, p10, p11) and (p00, p11, p01).
    Returns (nodes float64 [N, 3], tris int32 [K, 3]).
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    nodes = _NodeTable()
    tris = []
    for axis, sign, ua, va in _CUBE_FACES:
        ids = np.empty((n + 1, n + 1), dtype=np.int64)
        for a in range(n + 1):
            for b in range(n + 1):
                g = [0, 0, 0]
                g[axis] = sign * n
                g[ua] = 2 * a - n
                g[va] = 2 * b - n
                key = tuple(g)  # integer lattice in units of half / n
                xyz = [half * gi / n for gi in g]
                ids[a, b] = nodes.get(key, xyz)
        for a in range(n):
            for b in range(n):
                p00, p10, p11, p01 = ids[a, b], ids[a + 1, b], ids[a + 1, b + 1], ids[a, b + 1]
                tris.append((p00, p10, p11))
                tris.append((p00, p11, p01))
    return np.asarray(nodes.coords, dtype=np.float64), np.asarray(tris, dtype=np.int32)


def _red_refine(nodes: np.ndarray, tris: np.ndarray, project=None):
    """Split every triangle into 4 through its edge midpoints (shared between neighbours)."""
    nodes = [tuple(p) for p in nodes]
    mid = {}

    def midpoint(a, b):
        key = (a, b) if a < b else (b, a)
        nid = mid.get(key)
        if nid is None:
            p = [(nodes[a][k] + nodes[b][k]) * 0.5 for k in range(3)]
            if project is not None:
                p = project(p)
            nid = len(nodes)
            nodes.append(tuple(p))
            mid[key] = nid
        return nid

    out = []
    for a, b, c in tris.tolist():
        ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
        out += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
    return np.asarray(nodes, dtype=np.float64), np.asarray(out, dtype=np.int32)


def paper_cube(level: int = 1, half: float = 0.5):
    """Unit-cube family of Table 1: level 1 = 50 nodes / 96 elements, then red refinement."""
    if level < 1:
        raise ValueError("level must be >= 1")
    nodes = _NodeTable()
    tris = []
    m = 2  # squares per face edge
    for axis, sign, ua, va in _CUBE_FACES:
        def node(ga, gb, gn=None):
            g = [0, 0, 0]
            g[axis] = sign * 2 * m
            g[ua] = ga
            g[va] = gb
            key = tuple(g)  # lattice in units of half / (2 m)
            return nodes.get(key, [half * gi / (2 * m) for gi in g])

        for a in range(m):
            for b in range(m):
                # corners on the lattice -2m..2m in steps of 2, centre at odd offsets
                c00 = node(4 * a - 2 * m, 4 * b - 2 * m)
                c10 = node(4 * (a + 1) - 2 * m, 4 * b - 2 * m)
                c11 = node(4 * (a + 1) - 2 * m, 4 * (b + 1) - 2 * m)
                c01 = node(4 * a - 2 * m, 4 * (b + 1) - 2 * m)
                cc = node(4 * a + 2 - 2 * m, 4 * b + 2 - 2 * m)
                # counter-clockwise in (u, v) => normal along u x v (outward)
                tris += [(c00, c10, cc), (c10, c11, cc), (c11, c01, cc), (c01, c00, cc)]
    X = np.asarray(nodes.coords, dtype=np.float64)
    T = np.asarray(tris, dtype=np.int32)
    for _ in range(level - 1):
        X, T = _red_refine(X, T)
    return X, T


def icosphere(level: int = 3, radius: float = 1.0):
    """Icosahedron refined `level` times by edge midpoints projected onto the sphere."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
             (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
             (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]

    def project(p):
        nrm = math.sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2])
        return [radius * p[k] / nrm for k in range(3)]

    X = np.asarray([project(v) for v in verts], dtype=np.float64)
    T = np.asarray(faces, dtype=np.int32)
    for _ in range(level):
        X, T = _red_refine(X, T, project)
    # orient outward
    v0, v1, v2 = X[T[:, 0]], X[T[:, 1]], X[T[:, 2]]
    nrm = np.cross(v1 - v0, v2 - v0)
    flip = np.einsum("ij,ij->i", nrm, (v0 + v1 + v2)) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    return X, T


def bdf2_contour(L: int, dt: float = 0.1):
    """BDF2 gCQ contour points as a complex128 array of length L."""
    if L < 1:
        raise ValueError("L must be >= 1")
    R = 1e-10 ** (1.0 / (2 * L))
    ell = np.arange(L)
    z = R * np.exp(2j * np.pi * ell / L)
    s = (3.0 - 4.0 * z + z * z) / (2.0 * dt)
    # exact conjugate pairs: s_{L-l} = conj(s_l)
    for l in range(1, (L + 1) // 2):
        s[L - l] = np.conj(s[l])
    s[0] = s[0].real
    if L % 2 == 0:
        s[L // 2] = s[L // 2].real
    return s.astype(np.complex128)


def pulsating_sphere(points, normals, s, rho=1.0, cp=1.0, cs=0.5, a=2.5):
    """Exact displacement u and traction t = sigma n at points (normals n) of the radially
    pulsating unit sphere in the Laplace domain: u = A grad phi, phi = exp(-k r) / r,
    k = s / cp, scaled so that u(r = 1) = G(s) rh with G the Laplace transform of the pulse
    (a t)^4 exp(-a t) of Sec. 4.2 (a = 2.5); sigma from the isotropic stress law of
    Sec. 2.1.  Returns complex128 arrays [n, 3] (u, t)."""
    points = np.asarray(points, dtype=np.float64)
    normals = np.asarray(normals, dtype=np.float64)
    mu = rho * cs**2
    lam = rho * cp**2 - 2 * mu
    k = s / cp
    G = a**4 * 24.0 / (s + a) ** 5
    A = G / (-(1 + k) * np.exp(-k))
    r = np.linalg.norm(points, axis=1)
    rh = points / r[:, None]
    e = np.exp(-k * r)
    d1 = -(1 + k * r) * e / r**2
    d2 = (2 + 2 * k * r + (k * r) ** 2) * e / r**3
    u = (A * d1)[:, None] * rh
    rn = np.sum(rh * normals, axis=1)
    t = ((lam * A * k * k * e / r)[:, None] * normals
         + 2 * mu * A * ((d2 * rn)[:, None] * rh + (d1 / r)[:, None] * (normals - rn[:, None] * rh)))
    return u, t


def stator_shell(h: float = 0.05, r_out: float = 1.0, r_in: float = 0.7, length: float = 1.5,
                 n_slots: int = 36, slot_width: float = 0.05, slot_depth: float = 0.1):
    """Closed surface of an induction-machine-like stator: the solid between coaxial cylinders
    r = r_in and r = r_out, 0 <= z <= length, with n_slots slots (slot_width wide at the bore,
    slot_depth deep, radial walls) cut into the inner surface, and annular end caps; element
    size about h.  Cross-section: each sector holds a tooth (r_in <= r <= r_b = r_in +
    slot_depth between two slots, a structured grid whose side columns are the slot walls) and
    the annulus r_b <= r <= r_out above teeth and slot bottoms (a structured ring).  The side
    walls extrude the slotted inner contour and the outer circle.  Every edge is shared by two
    triangles; normals point out of the solid.  Returns (nodes [n, 3], tris [K, 3])."""
    S = n_slots
    dth = 2.0 * math.pi / S
    half = 0.5 * slot_width / r_in  # angular half-width of a slot at the bore
    r_b = r_in + slot_depth
    th0 = lambda k: k * dth + half          # tooth k from th0(k) to th1(k), slot k + 1 after it
    th1 = lambda k: (k + 1) * dth - half
    n_t = max(1, int(round(r_in * (th1(0) - th0(0)) / h)))
    n_w = max(1, int(round(slot_depth / h)))
    n_b = max(1, int(round(r_b * 2.0 * half / h)))
    n_r = max(1, int(round((r_out - r_b) / h)))
    n_z = max(1, int(round(length / h)))

    def canon(key):
        if key[0] == "b":  # slot bottom point i of the slot after tooth k
            _, k, i = key
            if i == 0:
                return ("g", k % S, n_t, n_w)
            if i == n_b:
                return ("g", (k + 1) % S, 0, n_w)
            return ("b", k % S, i)
        if key[0] == "g":
            return ("g", key[1] % S, key[2], key[3])
        return key

    def xy(key):
        if key[0] == "g":  # tooth grid: angle column a, radius level q
            _, k, a, q = key
            t = th0(k) + (th1(k) - th0(k)) * a / n_t
            r = r_in + slot_depth * q / n_w
        else:  # slot bottom
            _, k, i = key
            t = th1(k) + 2.0 * half * i / n_b
            r = r_b
        return r * math.cos(t), r * math.sin(t)

    # the slotted inner contour (counter-clockwise) and the ring at r_b
    contour, ring = [], []
    for k in range(S):
        contour += [canon(("g", k, a, 0)) for a in range(n_t)]
        contour += [canon(("g", k, n_t, q)) for q in range(n_w)]
        contour += [canon(("b", k, i)) for i in range(n_b)]
        contour += [canon(("g", k + 1, 0, q)) for q in range(n_w, 0, -1)]
        ring += [canon(("g", k, a, n_w)) for a in range(n_t)]
        ring += [canon(("b", k, i)) for i in range(n_b)]
    ring_th = [math.atan2(*reversed(xy(key))) for key in ring]
    nodes, idx = [], {}

    def node(key, p):
        if key not in idx:
            idx[key] = len(nodes)
            nodes.append(p)
        return idx[key]

    def plane(key, z, zi):
        """Node of a 2D key at height index zi (0 or n_z on the caps, interior on the walls)."""
        if key[0] == "o":
            t = ring_th[key[1]]
            p = (r_out * math.cos(t), r_out * math.sin(t))
        elif key[0] == "a":  # annulus level q between ring point i and the outer circle
            _, i, q = key
            t = ring_th[i]
            r = r_b + (r_out - r_b) * q / n_r
            p = (r * math.cos(t), r * math.sin(t))
        else:
            p = xy(key)
        return node((key, zi), (p[0], p[1], z))

    tris = []

    def quad(a, b, c, d, want):
        for t in ((a, b, c), (a, c, d)):
            P = [np.asarray(nodes[v]) for v in t]
            nrm = np.cross(P[1] - P[0], P[2] - P[0])
            tris.append(t if float(np.dot(nrm, want)) >= 0.0 else (t[0], t[2], t[1]))

    zs = np.linspace(0.0, length, n_z + 1)
    # inner side wall: outward normal of the solid = left of the counter-clockwise contour
    Mc = len(contour)
    for i in range(Mc):
        k0, k1 = contour[i], contour[(i + 1) % Mc]
        p0, p1 = np.asarray(xy(k0)), np.asarray(xy(k1))
        tg = p1 - p0
        want = np.array([-tg[1], tg[0], 0.0])
        for j in range(n_z):
            quad(plane(k0, zs[j], j), plane(k1, zs[j], j), plane(k1, zs[j + 1], j + 1), plane(k0, zs[j + 1], j + 1),
                 want)
    # outer side wall
    Mr = len(ring)
    for i in range(Mr):
        i1 = (i + 1) % Mr
        want = np.array([math.cos(ring_th[i]) + math.cos(ring_th[i1]), math.sin(ring_th[i]) + math.sin(ring_th[i1]), 0.0])
        for j in range(n_z):
            quad(plane(("o", i), zs[j], j), plane(("o", i1), zs[j], j), plane(("o", i1), zs[j + 1], j + 1),
                 plane(("o", i), zs[j + 1], j + 1), want)
    # caps: teeth and annulus at z = 0 (normal -z) and z = length (+z)
    for zi, z, sgn in ((0, 0.0, -1.0), (n_z, length, 1.0)):
        want = np.array([0.0, 0.0, sgn])
        for k in range(S):
            for a in range(n_t):
                for q in range(n_w):
                    quad(plane(canon(("g", k, a, q)), z, zi), plane(canon(("g", k, a + 1, q)), z, zi),
                         plane(canon(("g", k, a + 1, q + 1)), z, zi), plane(canon(("g", k, a, q + 1)), z, zi), want)
        lev = lambda i, q: ring[i] if q == 0 else (("o", i) if q == n_r else ("a", i, q))
        for i in range(Mr):
            i1 = (i + 1) % Mr
            for q in range(n_r):
                quad(plane(lev(i, q), z, zi), plane(lev(i1, q), z, zi), plane(lev(i1, q + 1), z, zi),
                     plane(lev(i, q + 1), z, zi), want)
    return np.asarray(nodes, dtype=np.float64), np.asarray(tris, dtype=np.int32)


def batch_meshes():
    """Meshes of the batched-product workload, smallest first: cubes [-1, 1]^3 with 8 and 16
    squares per face edge (768 and 3072 triangles) and icospheres of radius 1 with 1280 and
    5120 triangles.  Returns [(name, nodes, tris)]."""
    return [("cube768",) + cube_grid(8), ("sphere1280",) + icosphere(3),
            ("cube3072",) + cube_grid(16), ("sphere5120",) + icosphere(4)]


def random_rhs(seed: int, shape):
    """complex128 a + i b with a, b ~ N(0, 1) from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(shape)
    b = rng.standard_normal(shape)
    return (a + 1j * b).astype(np.complex128)


def mesh_summary(nodes: np.ndarray, tris: np.ndarray):
    """Counts and edge statistics used by tests and reports (no method arithmetic)."""
    edges = set()
    for a, b, c in tris.tolist():
        for p, q in ((a, b), (b, c), (c, a)):
            edges.add((p, q) if p < q else (q, p))
    return {"nodes": int(nodes.shape[0]), "elements": int(tris.shape[0]), "edges": len(edges)}
