"""Exact integrals of the Laplace Green's function over flat triangles.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.1 (discretisation paragraph) notes that for planar elements and
polynomial basis functions the boundary integrals can be taken analytically
instead of by quadrature.  For a flat triangle T with constant density 1
this module evaluates, at any point r off the triangle's edges,

    S(r)      = integral over T of 1 / |r - r'| dA'
    grad S(r) = - sum_e f_e m_e  -  W(r) n

where, for the edge e from vertex a to vertex b (counter-clockwise about the
unit normal n), t_e = (b - a)/|b - a| is its direction, m_e = t_e x n its
in-plane outward normal, and

    f_e  = integral along e of 1/|r - r'| ds'
         = asinh(s_b / d_e) - asinh(s_a / d_e),
           s_a = (a - r).t_e, s_b = (b - r).t_e, d_e = distance of r to the line of e,
    W(r) = integral over T of (r - r').n / |r - r'|^3 dA'
         = the solid angle T subtends at r, positive on the side n points to
           (zero for a point in the plane of T: the principal value).

The in-plane part of the gradient follows from the divergence theorem in the
plane of T (the boundary integral of 1/R times the outward normal), the
normal part from d/dh (1/R) = -h/R^3.  The potential is

    S(r) = sum_e P_e f_e - h W(r),   P_e = (a - r).m_e,  h = (r - a).n,

the contribution of each edge of the polar integral around the foot of r,
with the solid-angle term removing the part of the cone below the plane.
The solid angle is Van Oosterom and Strackee's closed form,
tan(W/2) = [R_1 . (R_2 x R_3)] / (R_1 R_2 R_3 + (R_1.R_2) R_3 + (R_1.R_3) R_2 + (R_2.R_3) R_1),
with R_k = v_k - r, taken with the opposite sign so that W has the sign of
h (seen from the side n points to, the vertices turn clockwise).

Dividing by 4 pi gives the single-layer potential of a unit density on T and
its gradient.  The pins (tests/test_oracle_panel_integrals.py) are an
adaptive one-dimensional polar quadrature of S, the closed form at the
centroid of an equilateral triangle, Gauss's law on a closed icosahedron for
W, central differences of S for grad S, and the point-source far-field limit.
"""
from __future__ import annotations

import numpy as np


def _edge_terms(v, r):
    """Per-edge (f_e, P_e, m_e) for triangle v (3, 3) and points r (M, 3)."""
    n = np.cross(v[1] - v[0], v[2] - v[0])
    n = n / np.linalg.norm(n)
    f = np.zeros((r.shape[0], 3))
    P = np.zeros((r.shape[0], 3))
    m = np.zeros((3, 3))
    for e in range(3):
        a, b = v[e], v[(e + 1) % 3]
        t = (b - a) / np.linalg.norm(b - a)
        me = np.cross(t, n)
        sa = (a - r) @ t
        sb = (b - r) @ t
        Ra = np.linalg.norm(a - r, axis=1)
        d2 = np.maximum(Ra * Ra - sa * sa, 0.0)
        d = np.sqrt(d2)
        with np.errstate(divide="ignore", invalid="ignore"):
            fe = np.arcsinh(sb / d) - np.arcsinh(sa / d)
            # on the line of the edge (outside the segment): log |s_b| / |s_a| with the sign of travel
            on_line = d <= 1e-14 * np.maximum(np.abs(sa), np.abs(sb))
            fe = np.where(on_line, np.sign(sb) * np.log(np.abs(sb) / np.abs(sa)), fe)
        f[:, e] = fe
        P[:, e] = (a - r) @ me
        m[e] = me
    return f, P, m, n


def solid_angle(v, r):
    """W(r): the solid angle T subtends at each point of r, signed, zero in
    the plane of T."""
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    R1, R2, R3 = v[0] - r, v[1] - r, v[2] - r
    l1, l2, l3 = (np.linalg.norm(x, axis=1) for x in (R1, R2, R3))
    # seen from the side n points to, the counter-clockwise vertices turn
    # clockwise, so the triple product of R_k = v_k - r is negative there
    num = -np.einsum("ij,ij->i", R1, np.cross(R2, R3))
    den = (l1 * l2 * l3 + np.einsum("ij,ij->i", R1, R2) * l3 + np.einsum("ij,ij->i", R1, R3) * l2
           + np.einsum("ij,ij->i", R2, R3) * l1)
    w = 2.0 * np.arctan2(num, den)
    # in the plane (num = 0): the principal value 0, also inside the triangle
    scale = l1 * l2 * l3
    return np.where(np.abs(num) <= 1e-15 * scale, 0.0, w)


def triangle_potential(v, r):
    """S(r) = integral over T of 1/|r - r'| dA' (v: (3, 3), r: (M, 3))."""
    v = np.asarray(v, dtype=np.float64)
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    f, P, m, n = _edge_terms(v, r)
    h = (r - v[0]) @ n
    return np.sum(P * f, axis=1) - h * solid_angle(v, r)


def triangle_grad(v, r):
    """grad_r S(r) (M, 3)."""
    v = np.asarray(v, dtype=np.float64)
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    f, P, m, n = _edge_terms(v, r)
    W = solid_angle(v, r)
    return -(f @ m) - W[:, None] * n[None, :]


def circumradius(verts, tris):
    """rho_j: the largest distance from panel j's centroid to its vertices."""
    V = np.asarray(verts, dtype=np.float64)[np.asarray(tris)]
    c = V.mean(axis=1)
    return np.linalg.norm(V - c[:, None, :], axis=2).max(axis=1)


def close_pairs(verts, tris, nu):
    """(i, j), i != j, with |c_i - c_j| < nu rho_j, sorted by (i, j): the
    panel pairs whose K' entry takes the exact integral over panel j."""
    from scipy.spatial import cKDTree

    V = np.asarray(verts, dtype=np.float64)[np.asarray(tris)]
    c = V.mean(axis=1)
    rho = circumradius(verts, tris)
    kd = cKDTree(c)
    out = []
    for j, nb in enumerate(kd.query_ball_point(c, nu * rho)):
        for i in nb:
            if i != j and np.sum((c[i] - c[j]) ** 2) < (nu * rho[j]) ** 2:
                out.append((i, j))
    out.sort()
    return np.array(out, dtype=np.int64).reshape(-1, 2)


def kprime_exact(verts, tris, normals, i, j):
    """K'_ij with the exact integral over panel j:
    n_i . grad_r of (1/4 pi) integral over T_j of 1/|r - r'| dA', at r = c_i."""
    V = np.asarray(verts, dtype=np.float64)[np.asarray(tris)]
    c = V.mean(axis=1)
    g = triangle_grad(V[j], c[i][None, :])[0]
    return float(np.dot(normals[i], g)) / (4.0 * np.pi)


def _correction_values(g, V, pairs):
    """exact - one-point K' of each close pair (i, j): n_i . grad of the
    single layer of panel j at c_i, less a_j n_i . grad G(c_i, c_j)."""
    delta = np.zeros(len(pairs))
    for k, (i, j) in enumerate(pairs):
        gi = triangle_grad(V[j], g.c[i][None, :])[0]
        exact = float(np.dot(g.n[i], gi)) / (4.0 * np.pi)
        d = g.c[i] - g.c[j]
        point = -g.a[j] * float(np.dot(g.n[i], d)) / (4.0 * np.pi * np.linalg.norm(d) ** 3)
        delta[k] = exact - point
    return delta


def kprime_correction(g, verts, tris, nu):
    """Sparse correction of K' for the near-quadrature operator: for every
    close pair (i, j) the difference between K'_ij with the exact integral
    over panel j and the one-point value a_j n_i . grad G(c_i, c_j).  Returns
    (rows, cols, delta), sorted by (row, col).  g: oracle Geometry of the
    same mesh (centroids, normals, areas)."""
    pairs = close_pairs(verts, tris, nu)
    if pairs.size == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0)
    V = np.asarray(verts, dtype=np.float64)[np.asarray(tris)]
    return pairs[:, 0], pairs[:, 1], _correction_values(g, V, pairs)


def kprime_correction_of(g, verts, tris, nu, panels, side="row"):
    """The entries of kprime_correction whose row (side="row": target panel)
    or column (side="col": source panel) is in `panels`, sorted by (row,
    col), for large meshes: the candidates come from a radius query about
    those panels' centroids (nu times the largest rho), then the same test
    |c_i - c_j| < nu rho_j and the same values as kprime_correction."""
    from scipy.spatial import cKDTree

    V = np.asarray(verts, dtype=np.float64)[np.asarray(tris)]
    c = V.mean(axis=1)
    rho = circumradius(verts, tris)
    kd = cKDTree(c)
    out = []
    for p in np.asarray(panels):
        for q in kd.query_ball_point(c[p], nu * rho.max()):
            i, j = (p, q) if side == "row" else (q, p)
            if i != j and np.sum((c[i] - c[j]) ** 2) < (nu * rho[j]) ** 2:
                out.append((i, j))
    out = sorted(set(out))
    pairs = np.array(out, dtype=np.int64).reshape(-1, 2)
    if pairs.size == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0)
    return pairs[:, 0], pairs[:, 1], _correction_values(g, V, pairs)


def apply_correction(corr, x, n, transpose=False):
    """sum over the close pairs (i, j) of delta_ij x_j into row i, or with
    transpose of delta_ij x_i into row j: the near-quadrature correction of
    K' x (or K'^T x), without the factor f of A."""
    rows, cols, delta = corr
    out = np.zeros(n)
    if transpose:
        np.add.at(out, cols, delta * x[rows])
    else:
        np.add.at(out, rows, delta * x[cols])
    return out


def apply_A_nq(g, f, x, corr):
    """A x with the near-quadrature K' (one-point elsewhere)."""
    from .dense import apply_A
    return apply_A(g, f, x) - f * apply_correction(corr, np.asarray(x, dtype=np.float64), g.N)


def apply_AT_nq(g, f, y, corr):
    """A^T y with the near-quadrature K'."""
    from .dense import apply_AT
    return apply_AT(g, f, y) - f * apply_correction(corr, np.asarray(y, dtype=np.float64), g.N, transpose=True)


def solve_nq(g, rq, q, eps_in, eps_out, corr):
    """x solving A x = f E with the near-quadrature A, by a LAPACK solve of
    the assembled matrix (small meshes)."""
    from .dense import assemble_A, f_factor, field_B
    f = f_factor(eps_in, eps_out)
    Am = assemble_A(g, f)
    rows, cols, delta = corr
    np.add.at(Am, (rows, cols), -f * delta)
    return np.linalg.solve(Am, f * field_B(g, rq, q))
