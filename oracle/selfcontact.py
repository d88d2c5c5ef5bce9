"""Self-collision rows: surface extraction, vertex-triangle detection and multi-node
contact rows (FP64; test infrastructure, like the rest of this package).

Paper: Sec. 6 (collision detection paragraph) states that the method handles self-contact
in principle because the contact Jacobian H may couple degrees of freedom of one object,
and leaves it off in its examples; Sec. 3.2 and App. A define a contact row as a
linearised constraint along a normal n and two tangents, delta_n = H_n q - d_n.  A
self-contact row is such a constraint on the gap between a surface vertex v and the point
p = sum_a w_a x_a of a surface triangle (barycentric weights w), so its Jacobian block is
C_j (e_v - sum_a w_a e_a) with C_j = (n, f1, f2) rows, and its Delassus entries are
K_jk = sum over the entries a of j and b of k of s_ja s_kb [A_n^-1]_(n_ja, n_kb), with
signs s = +1 for the vertex and -w_a for the triangle nodes.

Readings where the paper is silent:
* surface: the triangles that belong to exactly one tet, oriented so that their normal
  points away from the tet's fourth vertex;
* a pair (v, T) is a candidate iff v is a surface vertex that is not a corner of T;
  it is a contact iff, at x_t and at x~, the orthogonal projection of x_v onto the plane
  of T falls inside T (all barycentric weights >= 0), the signed distance along T's
  outward normal exceeds -margin at x_t (v is outside the body at the frame start up to
  the contact margin: an intersection-free state has every vertex outside, the band keeps
  a slightly penetrated vertex in contact, and it is far thinner than any wall, so the far
  side of the body never qualifies), v faces
  T at x_t (the sum of the area-weighted outward normals of v's surface triangles has a
  negative dot product with T's normal: the two surfaces are opposed, which excludes
  vertices next to a convex edge, whose projection falls on the perpendicular face just
  below its plane), and the smaller of the two states' distances is below margin (the
  obstacle predicate of the main contact model, applied to the triangle plane);
* the row's frame, weights and d_n are taken at x_t: n the outward unit normal of T,
  tangents as for obstacle rows, d_n = 0 (the gap is n . (x_v - p));
* canonical order: (vertex id, triangle id).

Pinned by the invariants in tests/test_oracle_selfcontact.py (closed-form geometry, a
hand-placed contact, balance of the pair, brute-force NCP solutions, and the frame loop's
momentum and non-penetration).
"""
from __future__ import annotations

import numpy as np

from .contact import tangent_basis

# faces of a tet (a, b, c, d) opposite each corner, with that corner last
_FACES = ((1, 2, 3, 0), (0, 3, 2, 1), (0, 1, 3, 2), (0, 2, 1, 3))


def surface_triangles(tets, rest):
    """Boundary triangles (m, 3) of a tet mesh, each oriented with its normal pointing away
    from the fourth vertex of its tet (outward), sorted by their sorted corner triple."""
    count, keep = {}, {}
    for t in np.asarray(tets, np.int64):
        for i, j, k, opp in _FACES:
            tri = [int(t[i]), int(t[j]), int(t[k])]
            a, b, c = (rest[x] for x in tri)
            if np.dot(np.cross(b - a, c - a), rest[int(t[opp])] - a) > 0.0:
                tri = [tri[0], tri[2], tri[1]]
            key = tuple(sorted(tri))
            count[key] = count.get(key, 0) + 1
            keep[key] = tri
    return np.array([keep[k] for k in sorted(count) if count[k] == 1], np.int64).reshape(-1, 3)


# Dot products and norms are written out component by component, summed left to right
# (x0 y0 + x1 y1) + x2 y2, so that their float64 rounding is fixed.
def _cross(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                     a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                     a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], axis=-1)


def _dot(a, b):
    return (a[..., 0] * b[..., 0] + a[..., 1] * b[..., 1]) + a[..., 2] * b[..., 2]


def triangle_frame(xa, xb, xc):
    """Outward unit normal of the triangle (a, b, c) and its area."""
    nrm = _cross(xb - xa, xc - xa)
    area2 = np.sqrt(_dot(nrm, nrm))
    return nrm / area2, 0.5 * area2


def project(x, xa, xb, xc):
    """Barycentric weights (w_a, w_b, w_c) of the orthogonal projection of x onto the
    plane of (a, b, c), and the signed distance of x along the outward normal."""
    n, _ = triangle_frame(xa, xb, xc)
    dist = float(_dot(n, x - xa))
    p = x - dist * n
    # areas of the sub-triangles opposite each corner, signed by the normal
    wa = _dot(n, _cross(xb - p, xc - p))
    wb = _dot(n, _cross(xc - p, xa - p))
    wc = _dot(n, _cross(xa - p, xb - p))
    tot = (wa + wb) + wc
    return np.array([wa, wb, wc]) / tot, dist


def vertex_normals(x, tris):
    """Sum over each vertex's surface triangles of their area-weighted outward normals
    (the cross product of two edges), at positions x; zero for non-surface vertices."""
    out = np.zeros_like(np.asarray(x, np.float64))
    for a, b, c in tris:  # in triangle order
        nrm = _cross(x[b] - x[a], x[c] - x[a])
        out[a] += nrm
        out[b] += nrm
        out[c] += nrm
    return out


def detect_self(q_t, q_pred, tris, margin):
    """Vertex-triangle self-contacts: list of (v, triangle index) in canonical order.

    Each vertex is tested against every triangle (vectorised over triangles)."""
    tris = np.asarray(tris, np.int64).reshape(-1, 3)
    verts = np.unique(tris)
    vn = vertex_normals(q_t, tris)
    geo = []
    for q in (q_t, q_pred):
        xa, xb, xc = q[tris[:, 0]], q[tris[:, 1]], q[tris[:, 2]]
        nrm = _cross(xb - xa, xc - xa)
        nrm = nrm / np.sqrt(_dot(nrm, nrm))[:, None]
        geo.append((xa, xb, xc, nrm))
    out = []
    for v in verts:
        keep = ~np.any(tris == v, axis=1) & (_dot(geo[0][3], vn[v][None, :]) < 0.0)
        dists = []
        for q, (xa, xb, xc, nrm) in zip((q_t, q_pred), geo):
            x = q[v]
            dist = _dot(nrm, x[None, :] - xa)
            p = x - dist[:, None] * nrm
            wa = _dot(nrm, _cross(xb - p, xc - p))
            wb = _dot(nrm, _cross(xc - p, xa - p))
            wc = _dot(nrm, _cross(xa - p, xb - p))
            tot = (wa + wb) + wc
            keep &= (wa / tot >= 0.0) & (wb / tot >= 0.0) & (wc / tot >= 0.0)
            dists.append(dist)
        keep &= (dists[0] > -margin) & (np.minimum(dists[0], dists[1]) < margin)
        out.extend((int(v), int(ti)) for ti in np.flatnonzero(keep))
    return out


class SelfRows:
    """Multi-node contact rows at x_t: entries (nodes, signs), frames C (c, 3, 3)."""

    def __init__(self, pairs, tris, q_t):
        c = len(pairs)
        self.nodes = np.zeros((c, 4), np.int64)
        self.signs = np.zeros((c, 4))
        self.C = np.zeros((c, 3, 3))
        self.gap = np.zeros(c)
        for j, (v, ti) in enumerate(pairs):
            tri = tris[ti]
            w, dist = project(q_t[v], q_t[tri[0]], q_t[tri[1]], q_t[tri[2]])
            n, _ = triangle_frame(q_t[tri[0]], q_t[tri[1]], q_t[tri[2]])
            f1, f2 = tangent_basis(n)
            self.nodes[j] = [v, tri[0], tri[1], tri[2]]
            self.signs[j] = [1.0, -w[0], -w[1], -w[2]]
            self.C[j] = np.stack([n, f1, f2])
            self.gap[j] = dist

    @property
    def c(self):
        return len(self.nodes)

    def H(self, n):
        """Dense contact Jacobian (3c, 3n): block (j, node) = s C_j, node-major columns."""
        Hm = np.zeros((3 * self.c, 3 * n))
        for j in range(self.c):
            for a in range(4):
                v = self.nodes[j, a]
                Hm[3 * j:3 * j + 3, 3 * v:3 * v + 3] += self.signs[j, a] * self.C[j]
        return Hm

    def H_T(self, lam, n):
        """Nodal forces (n, 3) of per-row components lam (c, 3): sum of s C_j^T lam_j."""
        out = np.zeros((n, 3))
        for j in range(self.c):
            f = self.C[j].T @ lam[j]
            for a in range(4):
                out[self.nodes[j, a]] += self.signs[j, a] * f
        return out

    def delassus(self, solve, n):
        """K_jk = sum_a sum_b s_ja s_kb [A_n^-1]_(n_ja, n_kb), the columns of A_n^-1 by
        solves with `solve` (n x m right-hand sides); W = K_jk C_j C_k^T blocks."""
        c = self.c
        if c == 0:
            return np.zeros((0, 0)), np.zeros((0, 0))
        B = np.zeros((n, c))
        for j in range(c):
            for a in range(4):
                B[self.nodes[j, a], j] += self.signs[j, a]
        Z = solve(B)
        K = B.T @ Z
        K = 0.5 * (K + K.T)
        W = np.einsum("jk,jab,kcb->jakc", K, self.C, self.C).reshape(3 * c, 3 * c)
        return K, W
