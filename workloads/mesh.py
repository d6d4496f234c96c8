"""Seeded structured meshes, face tables and canonical face frames (input generator).

The paper's meshes are not available; these are synthetic stand-ins with the
shapes of its workloads. Faces are numbered by first appearance while looping
over elements and their local faces, so e1 < e2 on every interior face.

Face orientation (not specified by the paper): every face gets a canonical
parameterisation derived from the global vertex ids of its corners, which both
neighbouring elements reproduce, so trace dofs need no permutation.
"""
import numpy as np

# Reference vertices in [0,1]^d; tensor cells list vertices with x fastest.
REF_VERTS = {
    "quad": np.array([[0, 0], [1, 0], [0, 1], [1, 1]], float),
    "hex": np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], float),
    "tri": np.array([[0, 0], [1, 0], [0, 1]], float),
    "tet": np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float),
}
# Local faces as lists of local vertices (tensor cells: face corners in tensor order).
LOCAL_FACES = {
    "quad": [(0, 2), (1, 3), (0, 1), (2, 3)],
    "hex": [(0, 2, 4, 6), (1, 3, 5, 7), (0, 1, 4, 5), (2, 3, 6, 7), (0, 1, 2, 3), (4, 5, 6, 7)],
    "tri": [(1, 2), (0, 2), (0, 1)],
    "tet": [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)],
}
DIM = {"quad": 2, "hex": 3, "tri": 2, "tet": 3}


class Mesh:
    def __init__(self, etype, verts, elems):
        self.etype = etype
        self.dim = DIM[etype]
        self.verts = np.ascontiguousarray(verts, dtype=np.float64)
        self.elems = np.ascontiguousarray(elems, dtype=np.int64)
        self.ne = self.elems.shape[0]
        self.nlfe = len(LOCAL_FACES[etype])
        self._build_faces()

    def _build_faces(self):
        lf = LOCAL_FACES[self.etype]
        table = {}
        f2e = []
        e2f = np.zeros((self.ne, self.nlfe), np.int64)
        for e in range(self.ne):
            ev = self.elems[e]
            for l, loc in enumerate(lf):
                key = tuple(sorted(int(ev[v]) for v in loc))
                f = table.get(key)
                if f is None:
                    f = len(f2e)
                    table[key] = f
                    f2e.append([e, l, -1, -1])
                else:
                    assert f2e[f][2] < 0, "face shared by more than two elements"
                    f2e[f][2] = e
                    f2e[f][3] = l
                e2f[e, l] = f
        self.f2e = np.array(f2e, np.int64)
        self.e2f = e2f
        self.nf = self.f2e.shape[0]
        self.boundary = self.f2e[:, 2] < 0

    def face_frame(self, e, l):
        """Affine map of the canonical face parameter domain into element e's
        reference cell: xi = o + s*a (+ t*b). Returns (o, A) with A columns a, b."""
        et = self.etype
        loc = LOCAL_FACES[et][l]
        gid = [int(self.elems[e][v]) for v in loc]
        R = REF_VERTS[et]
        if et in ("quad", "tri"):
            i0, i1 = (0, 1) if gid[0] < gid[1] else (1, 0)
            o = R[loc[i0]]
            return o, (R[loc[i1]] - o)[:, None]
        if et == "hex":
            k0 = int(np.argmin(gid))
            nb = [k0 ^ 1, k0 ^ 2]
            if gid[nb[0]] > gid[nb[1]]:
                nb = nb[::-1]
            o = R[loc[k0]]
            return o, np.stack([R[loc[nb[0]]] - o, R[loc[nb[1]]] - o], axis=1)
        if et == "tet":
            order = np.argsort(gid)
            o = R[loc[order[0]]]
            return o, np.stack([R[loc[order[1]]] - o, R[loc[order[2]]] - o], axis=1)
        raise ValueError(et)

    def face_frames(self):
        """(ne, nlfe, dim) origins and (ne, nlfe, dim, dim-1) axes for all local faces."""
        O = np.zeros((self.ne, self.nlfe, self.dim))
        A = np.zeros((self.ne, self.nlfe, self.dim, self.dim - 1))
        for e in range(self.ne):
            for l in range(self.nlfe):
                O[e, l], A[e, l] = self.face_frame(e, l)
        return O, A


def _jitter(verts, interior, h, amp, seed):
    rng = np.random.default_rng(seed)
    d = rng.uniform(-amp * h, amp * h, size=verts.shape)
    verts = verts.copy()
    verts[interior] += d[interior]
    return verts


def _grid(n, dim):
    ax = np.arange(n + 1) / n
    g = np.meshgrid(*([ax] * dim), indexing="ij")
    verts = np.stack([x.transpose().reshape(-1) for x in g], axis=1)   # x fastest
    interior = np.all((verts > 1e-12) & (verts < 1 - 1e-12), axis=1)
    return verts, interior


def structured_quads(n, amp=0.0, seed=0):
    verts, interior = _grid(n, 2)
    verts = _jitter(verts, interior, 1.0 / n, amp, seed)
    vid = lambda i, j: j * (n + 1) + i
    elems = [[vid(i, j), vid(i + 1, j), vid(i, j + 1), vid(i + 1, j + 1)]
             for j in range(n) for i in range(n)]
    return Mesh("quad", verts, elems)


def structured_hexes(n, amp=0.0, seed=0):
    verts, interior = _grid(n, 3)
    verts = _jitter(verts, interior, 1.0 / n, amp, seed)
    vid = lambda i, j, k: (k * (n + 1) + j) * (n + 1) + i
    elems = []
    for k in range(n):
        for j in range(n):
            for i in range(n):
                elems.append([vid(i + (c & 1), j + ((c >> 1) & 1), k + ((c >> 2) & 1)) for c in range(8)])
    return Mesh("hex", verts, elems)


def structured_tris(n, amp=0.0, seed=0):
    """n x n squares, each cut along the (0,0)-(1,1) diagonal into two triangles."""
    verts, interior = _grid(n, 2)
    verts = _jitter(verts, interior, 1.0 / n, amp, seed)
    vid = lambda i, j: j * (n + 1) + i
    elems = []
    for j in range(n):
        for i in range(n):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i, j + 1), vid(i + 1, j + 1)
            elems.append([a, b, d])
            elems.append([a, d, c])
    return Mesh("tri", verts, elems)


def kuhn_tets(n, amp=0.0, seed=0):
    """n^3 cubes, each split into the 6 Kuhn tetrahedra along the main diagonal."""
    verts, interior = _grid(n, 3)
    verts = _jitter(verts, interior, 1.0 / n, amp, seed)
    vid = lambda i, j, k: (k * (n + 1) + j) * (n + 1) + i
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    elems = []
    for k in range(n):
        for j in range(n):
            for i in range(n):
                for pm in perms:
                    c = [0, 0, 0]
                    path = [vid(i, j, k)]
                    for ax in pm:
                        c[ax] += 1
                        path.append(vid(i + c[0], j + c[1], k + c[2]))
                    elems.append(path)
    m = Mesh("tet", verts, elems)
    # orient every tet positively (swap two vertices where needed)
    X = m.verts[m.elems]
    vol = np.einsum("ij,ij->i", np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]), X[:, 3] - X[:, 0])
    neg = vol < 0
    if np.any(neg):
        el = m.elems.copy()
        el[neg, 1], el[neg, 2] = m.elems[neg, 2], m.elems[neg, 1]
        m = Mesh("tet", m.verts, el)
    return m


def reference_map(etype, X, xi):
    """Physical points and Jacobians. X (ne, nv, dim) element vertices, xi (nq, dim).

    Returns x (ne, nq, dim) and J (ne, nq, dim, dim) with J[..., i, j] = dx_i/dxi_j.
    """
    dim = X.shape[2]
    if etype in ("tri", "tet"):
        A = np.stack([X[:, k + 1] - X[:, 0] for k in range(dim)], axis=2)   # (ne, dim, dim)
        x = X[:, None, 0, :] + np.einsum("eij,qj->eqi", A, xi)
        J = np.broadcast_to(A[:, None], (X.shape[0], xi.shape[0], dim, dim)).copy()
        return x, J
    nv = 2 ** dim
    N = np.ones((xi.shape[0], nv))
    dN = np.ones((xi.shape[0], nv, dim))
    for v in range(nv):
        bits = [(v >> d) & 1 for d in range(dim)]
        for d in range(dim):
            f = xi[:, d] if bits[d] else 1 - xi[:, d]
            df = 1.0 if bits[d] else -1.0
            N[:, v] *= f
            for g in range(dim):
                dN[:, v, g] *= (df if g == d else f)
    x = np.einsum("qv,evi->eqi", N, X)
    J = np.einsum("qvj,evi->eqij", dN, X)
    return x, J
