"""Macro meshes, structured refinement, node sets and the blending map.

Follows Sec. 4.1 ("Mesh and Blending") and Sec. 4.2 of arXiv 2506.04157:

* an unstructured coarse grid of tetrahedra ("macro-tetrahedra") is refined
  uniformly and structurally (Bey's scheme), every macro-tet into 8^L
  micro-tets at level L;
* the hollow sphere is built from the hollow icosahedron: each triangular
  face is subdivided, each small triangle spans a truncated pyramid (prism)
  between two spheres, the prisms are cut into radial layers of equal
  height, and each prism is cut into three tetrahedra;
* the refined reference mesh is mapped to the physical domain by a blending
  map B that is C^0 globally and smooth on every macro-tet;
* P2 velocity nodes are the vertices and edge midpoints of the *reference*
  (unblended) micro-tets; P1 nodes are the vertices.

Readings where the paper is silent (they are stated by specification and
implemented independently on the GPU side):

* icosahedron vertices: the cyclic permutations of (0, +-1, +-phi),
  normalised, in the order listed in ``icosahedron_vertices``;
* face subdivision: uniform in the flat face, points projected to the sphere;
  each sphere point is identified by its integer weight vector over the 12
  icosahedron vertices, and points are totally ordered by lexicographic
  order of that vector;
* prism split: with the triangle's sphere points sorted v0 < v1 < v2 and
  a_i (inner) / b_i (outer) the prism corners, the tetrahedra are
  (a0,a1,a2,b2), (a0,a1,b1,b2), (a0,b0,b1,b2) (every quadrilateral side is
  cut from the inner corner of its smaller point to the outer corner of its
  larger point, so neighbouring prisms agree);
* the octahedron left in the middle of Bey's refinement step is cut along
  the lattice diagonal b <-> a+c;
* blending: B(x) = s(x) x/|x| with s the affine interpolant of the vertex
  radii over the macro-tet; the unit cube uses B = id.
"""
from itertools import permutations

import numpy as np

PHI = (1.0 + 5.0 ** 0.5) / 2.0


# ---------------------------------------------------------------------------
# macro meshes
# ---------------------------------------------------------------------------

def icosahedron_vertices():
    """The 12 unit icosahedron vertices in the fixed order used by the mesh."""
    raw = [
        (0.0, 1.0, PHI), (0.0, -1.0, PHI), (0.0, 1.0, -PHI), (0.0, -1.0, -PHI),
        (1.0, PHI, 0.0), (-1.0, PHI, 0.0), (1.0, -PHI, 0.0), (-1.0, -PHI, 0.0),
        (PHI, 0.0, 1.0), (-PHI, 0.0, 1.0), (PHI, 0.0, -1.0), (-PHI, 0.0, -1.0),
    ]
    v = np.array(raw)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def icosahedron_faces():
    """The 20 faces as sorted vertex triples (mutually adjacent vertices)."""
    v = icosahedron_vertices()
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    edge = d.min(where=d > 1e-9, initial=10.0)
    adj = np.abs(d - edge) < 1e-9
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            for k in range(j + 1, 12):
                if adj[i, j] and adj[j, k] and adj[i, k]:
                    faces.append((i, j, k))
    assert len(faces) == 20
    return faces


class MacroMesh:
    """Coarse tetrahedral mesh.

    vertices : (nv, 3) reference coordinates
    tets     : (nm, 4) vertex ids; the vertex order defines the refinement
    layer    : (nv,) radial layer index (shell) or -1 (cube)
    """

    def __init__(self, kind, vertices, tets, layer, r_in=None, r_out=None,
                 n_rad=None):
        self.kind = kind
        self.vertices = np.asarray(vertices, dtype=np.float64)
        self.tets = np.asarray(tets, dtype=np.int64)
        self.layer = np.asarray(layer, dtype=np.int64)
        self.r_in, self.r_out, self.n_rad = r_in, r_out, n_rad

    @property
    def n_macros(self):
        return len(self.tets)


def cube_macros():
    """Unit cube as six tetrahedra along the Kuhn paths 0 -> e_s1 -> e_s1+e_s2 -> 1."""
    corners = np.array([[x, y, z] for x in (0, 1) for y in (0, 1) for z in (0, 1)],
                       dtype=np.float64)
    cid = {tuple(c.astype(int)): i for i, c in enumerate(corners)}
    tets = []
    for s in permutations(range(3)):
        p = np.zeros(3, dtype=int)
        path = [cid[tuple(p)]]
        for ax in s:
            p = p.copy()
            p[ax] = 1
            path.append(cid[tuple(p)])
        tets.append(path)
    return MacroMesh("cube", corners, tets, -np.ones(8, dtype=np.int64))


def shell_macros(n_tan, n_rad, r_in, r_out):
    """Icosahedral hollow-sphere macro mesh: 60 n_tan^2 n_rad macro-tets."""
    ico = icosahedron_vertices()
    faces = icosahedron_faces()
    keys, tris = [], []
    for (I, J, K) in faces:
        idx = {}
        for i in range(n_tan + 1):
            for j in range(n_tan + 1 - i):
                w = np.zeros(12, dtype=np.int64)
                w[I] += i
                w[J] += j
                w[K] += n_tan - i - j
                idx[(i, j)] = len(keys)
                keys.append(w)
        for i in range(n_tan):
            for j in range(n_tan - i):
                tris.append((idx[(i, j)], idx[(i + 1, j)], idx[(i, j + 1)]))
                if i + j <= n_tan - 2:
                    tris.append((idx[(i + 1, j)], idx[(i, j + 1)], idx[(i + 1, j + 1)]))
    keys = np.array(keys)
    # np.unique sorts rows lexicographically: the point id *is* the key rank
    ukeys, inv = np.unique(keys, axis=0, return_inverse=True)
    inv = inv.ravel()
    tris = inv[np.array(tris)]
    dirs = ukeys.astype(np.float64) @ ico
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    ns = len(ukeys)
    radii = r_in + (r_out - r_in) * np.arange(n_rad + 1) / n_rad
    verts = np.concatenate([r * dirs for r in radii])
    layer = np.repeat(np.arange(n_rad + 1), ns)
    tets = []
    for t in tris:
        s0, s1, s2 = np.sort(t)
        for k in range(n_rad):
            a = [s0 + k * ns, s1 + k * ns, s2 + k * ns]
            b = [s0 + (k + 1) * ns, s1 + (k + 1) * ns, s2 + (k + 1) * ns]
            tets.append((a[0], a[1], a[2], b[2]))
            tets.append((a[0], a[1], b[1], b[2]))
            tets.append((a[0], b[0], b[1], b[2]))
    return MacroMesh("shell", verts, tets, layer, r_in, r_out, n_rad)


# ---------------------------------------------------------------------------
# structured refinement of one macro-tet (lattice description)
# ---------------------------------------------------------------------------

EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def lattice_points(m):
    """All (i, j, k) with i + j + k <= m, as an (np, 3) int array."""
    pts = [(i, j, k) for k in range(m + 1) for j in range(m + 1 - k)
           for i in range(m + 1 - j - k)]
    return np.array(pts, dtype=np.int64)


def micro_tets(n):
    """Micro-tets of a macro refined to n = 2^L, as (n^3, 4, 3) P1 lattice coords.

    Up tets p+{0,a,b,c}; octahedra p+{a,b,c,a+b,a+c,b+c} cut along b <-> a+c
    into four tets; down tets p+{a+b,a+c,b+c,a+b+c}.
    """
    a, b, c = np.eye(3, dtype=np.int64)
    out = []
    for p in lattice_points(n - 1):
        out.append([p, p + a, p + b, p + c])
    if n >= 2:
        for p in lattice_points(n - 2):
            A, Bv, Cv = p + a, p + b, p + c
            AB, AC, BC = p + a + b, p + a + c, p + b + c
            out.append([Bv, AC, A, AB])
            out.append([Bv, AC, AB, BC])
            out.append([Bv, AC, BC, Cv])
            out.append([Bv, AC, Cv, A])
    if n >= 3:
        for p in lattice_points(n - 3):
            out.append([p + a + b, p + a + c, p + b + c, p + a + b + c])
    out = np.array(out, dtype=np.int64).reshape(-1, 4, 3)
    assert len(out) == n ** 3
    return out


# ---------------------------------------------------------------------------
# refined mesh with global node numbering
# ---------------------------------------------------------------------------

def _node_keys(gids, weights):
    """Canonical integer key of lattice points: (vertex id, weight) pairs
    sorted by vertex id, zero weights dropped (padded with -1, 0)."""
    g = np.where(weights > 0, gids, np.iinfo(np.int64).max)
    order = np.argsort(g, axis=-1, kind="stable")
    gs = np.take_along_axis(g, order, axis=-1)
    ws = np.take_along_axis(weights, order, axis=-1)
    gs = np.where(gs == np.iinfo(np.int64).max, -1, gs)
    return np.concatenate([gs, ws], axis=-1)


class RefinedMesh:
    """Refined mesh at one level.

    Attributes
    ----------
    x2, x1      reference coordinates of P2 / P1 nodes
    X2, X1      physical (blended) coordinates
    e2          (ne, 10) P2 node ids per element: vertices 0..3 then edges
                01, 02, 03, 12, 13, 23
    e1          (ne, 4) P1 node ids per element
    emacro      (ne,) macro id of each element
    ev          (ne, 4, 3) reference vertex coordinates per element
    """

    def __init__(self, macro, level):
        self.macro = macro
        self.level = level
        n = 2 ** level
        self.n = n
        mt = micro_tets(n)                       # (ne_loc, 4, 3)
        ne_loc = len(mt)
        tets = macro.tets                        # (nm, 4)
        nm = len(tets)
        # barycentric integer weights of the 4 element vertices on the P1 lattice
        w1 = np.concatenate([n - mt.sum(-1, keepdims=True), mt], axis=-1)   # (ne_loc,4,4)
        # P2 lattice: vertices doubled, edges summed
        w2v = 2 * w1
        w2e = np.stack([w1[:, i] + w1[:, j] for (i, j) in EDGES], axis=1)
        w2 = np.concatenate([w2v, w2e], axis=1)                              # (ne_loc,10,4)
        gid = tets[:, None, None, :]                                          # (nm,1,1,4)
        k2 = _node_keys(np.broadcast_to(gid, (nm, ne_loc, 10, 4)),
                        np.broadcast_to(w2[None], (nm, ne_loc, 10, 4)))
        k2 = k2.reshape(-1, 8)
        u2, inv2 = np.unique(k2, axis=0, return_inverse=True)
        self.e2 = inv2.ravel().reshape(nm * ne_loc, 10)
        k1 = _node_keys(np.broadcast_to(gid, (nm, ne_loc, 4, 4)),
                        np.broadcast_to(w1[None], (nm, ne_loc, 4, 4)))
        u1, inv1 = np.unique(k1.reshape(-1, 8), axis=0, return_inverse=True)
        self.e1 = inv1.ravel().reshape(nm * ne_loc, 4)
        self.emacro = np.repeat(np.arange(nm), ne_loc)
        V = macro.vertices
        self.x2 = self._coords(u2, V, 2 * n)
        self.x1 = self._coords(u1, V, n)
        mv = V[tets]                                                          # (nm,4,3)
        ev = np.einsum("lvk,mkd->mlvd", w1.astype(np.float64) / n, mv)
        self.ev = ev.reshape(nm * ne_loc, 4, 3)
        self.keys2, self.keys1 = u2, u1
        # blending constants per macro: s(x) = g.x + s0 interpolates |v_i|
        if macro.kind == "shell":
            A = np.concatenate([mv, np.ones((nm, 4, 1))], axis=2)
            rad = np.linalg.norm(mv, axis=2)
            sol = np.linalg.solve(A, rad[..., None])[..., 0]
            self.blend_g = sol[:, :3]
            self.blend_s0 = sol[:, 3]
        else:
            self.blend_g = None
            self.blend_s0 = None
        # physical coordinates: blend with the macro of any element holding the node
        self.X2 = self.blend_points(self.x2, self._node_macro(self.e2, len(u2)))
        self.X1 = self.blend_points(self.x1, self._node_macro(self.e1, len(u1)))
        self._classify(u2, u1)

    # -- helpers -----------------------------------------------------------
    @staticmethod
    def _coords(keys, V, m):
        gs, ws = keys[:, :4], keys[:, 4:]
        gs = np.where(gs < 0, 0, gs)
        return np.einsum("pk,pkd->pd", ws / m, V[gs])

    def _node_macro(self, enodes, nn):
        out = np.empty(nn, dtype=np.int64)
        out[enodes.ravel()] = np.repeat(self.emacro, enodes.shape[1])
        return out

    def blend_points(self, xt, macro_ids):
        """B(x~) = s(x~) x~/|x~| with s affine per macro (identity for the cube)."""
        if self.blend_g is None:
            return xt.copy()
        s = np.einsum("pd,pd->p", self.blend_g[macro_ids], xt) + self.blend_s0[macro_ids]
        return xt * (s / np.linalg.norm(xt, axis=1))[:, None]

    def _classify(self, u2, u1):
        """Boundary flags: 1 = inner sphere / cube boundary, 2 = outer sphere."""
        mac = self.macro
        if mac.kind == "shell":
            def flags(keys):
                gs, ws = keys[:, :4], keys[:, 4:]
                lay = np.where(ws > 0, mac.layer[np.where(gs < 0, 0, gs)], -7)
                inner = np.all((lay == 0) | (ws == 0), axis=1)
                outer = np.all((lay == mac.n_rad) | (ws == 0), axis=1)
                return inner.astype(np.int8) + 2 * outer.astype(np.int8)
            self.flag2 = flags(u2)
            self.flag1 = flags(u1)
        else:
            def flags(x):
                on = np.any((x == 0.0) | (x == 1.0), axis=1)
                return on.astype(np.int8)
            self.flag2 = flags(self.x2)
            self.flag1 = flags(self.x1)

    @property
    def n2(self):
        return len(self.x2)

    @property
    def n1(self):
        return len(self.x1)

    @property
    def ne(self):
        return len(self.e2)


def kuhn_cube(level):
    """The unit cube split directly into the Kuhn (Freudenthal) grid.

    Independent construction used to pin the structured refinement: each of
    the (2^L)^3 grid cubes is cut into the six tets c, c+e_s1, c+e_s1+e_s2, c+1.
    Returns (x2, e2, x1, e1) with the same local node order as RefinedMesh.
    """
    N = 2 ** level
    M = 2 * N + 1
    lin2 = lambda p: (p[..., 0] * M + p[..., 1]) * M + p[..., 2]
    cells = np.array([(i, j, k) for i in range(N) for j in range(N) for k in range(N)])
    tets = []
    for s in permutations(range(3)):
        path = [np.zeros(3, dtype=int)]
        for ax in s:
            q = path[-1].copy()
            q[ax] += 1
            path.append(q)
        tets.append(np.array(path))
    tets = np.array(tets)                                   # (6,4,3)
    verts = cells[:, None, None, :] + tets[None]           # (nc,6,4,3)
    verts = verts.reshape(-1, 4, 3)
    p2v = 2 * verts
    p2e = np.stack([verts[:, i] + verts[:, j] for (i, j) in EDGES], axis=1)
    p2 = np.concatenate([p2v, p2e], axis=1)
    g = np.stack(np.meshgrid(np.arange(M), np.arange(M), np.arange(M), indexing="ij"), -1)
    x2 = g.reshape(-1, 3) / (2 * N)
    e2 = lin2(p2)
    M1 = N + 1
    g1 = np.stack(np.meshgrid(np.arange(M1), np.arange(M1), np.arange(M1), indexing="ij"), -1)
    x1 = g1.reshape(-1, 3) / N
    e1 = (verts[..., 0] * M1 + verts[..., 1]) * M1 + verts[..., 2]
    return x2, e2, x1, e1


# ---------------------------------------------------------------------------
# node / DoF counts
# ---------------------------------------------------------------------------

def shell_counts(n_tan, n_rad, level):
    """Closed-form P2 and P1 node counts of the icosahedral shell.

    With N = n_tan 2^L points per icosahedron edge and M = n_rad 2^L radial
    intervals, the sphere holds 10 N^2 + 2 points.
    """
    N = n_tan * 2 ** level
    M = n_rad * 2 ** level
    return (10 * (2 * N) ** 2 + 2) * (2 * M + 1), (10 * N ** 2 + 2) * (M + 1)
