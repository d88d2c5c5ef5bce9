"""Pins of the self-contact oracle (oracle/selfcontact.py) against geometry and mechanics
that fix its results independently: closed-form surfaces and barycentric coordinates,
hand-placed contacts, Newton's third law and zero torque of the contact pair, and the
Delassus block against the dense product H (A_n (x) I3)^-1 H^T."""
import numpy as np
import pytest

from oracle import selfcontact as scx
from paper_2503_15078_amd import scenes

# two separate tets: the top one's lowest vertex (4) hovers 0.005 above the bottom one's
# upward face (0, 1, 2), over the point (0.2, 0.2, 0)
STACK = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, -1],
                  [0.2, 0.2, 0.005], [0.2, 0.2, 1], [1, 0.2, 1], [0.2, 1, 1]], float)
STACK_TETS = np.array([[0, 1, 2, 3], [4, 5, 6, 7]])


def test_single_tet_surface_is_outward():
    X = STACK[:4]
    tris = scx.surface_triangles(STACK_TETS[:1], X)
    assert len(tris) == 4
    centre = X.mean(0)
    for t in tris:
        n, _ = scx.triangle_frame(*X[t])
        assert np.dot(n, X[t].mean(0) - centre) > 0.0


def test_one_voxel_cube_surface():
    """Five-tet split of a cube: 20 tet faces, 4 interior (shared), 12 on the boundary,
    covering the six square faces (area 6 e^2), all outward."""
    sc = scenes.cube_drop(0, nodes=2)
    tris = scx.surface_triangles(sc.tets, sc.rest)
    assert len(tris) == 12
    e = np.ptp(sc.rest[:, 0])
    centre = sc.rest.mean(0)
    area = 0.0
    for t in tris:
        n, a = scx.triangle_frame(*sc.rest[t])
        area += a
        assert np.dot(n, sc.rest[t].mean(0) - centre) > 0.0
    assert area == pytest.approx(6.0 * e * e, rel=1e-12)


def test_projection_closed_forms():
    a, b, c = np.array([0.0, 0, 0]), np.array([1.0, 0, 0]), np.array([0.0, 1, 0])
    w, d = scx.project(np.array([1 / 3, 1 / 3, 0.2]), a, b, c)
    np.testing.assert_allclose(w, [1 / 3, 1 / 3, 1 / 3], atol=1e-15)
    assert d == pytest.approx(0.2)
    w, d = scx.project(np.array([0.5, 0.5, -0.1]), a, b, c)
    np.testing.assert_allclose(w, [0.0, 0.5, 0.5], atol=1e-15)
    assert d == pytest.approx(-0.1)
    w, _ = scx.project(np.array([1.0, 1.0, 0.0]), a, b, c)
    assert w[0] == pytest.approx(-1.0) and w.sum() == pytest.approx(1.0)


def test_convex_body_at_rest_has_no_self_contacts():
    """Every vertex touches its own triangles (excluded) and lies a full edge inside the
    opposite faces (further inside than the margin), so a convex cube at rest has none."""
    sc = scenes.cube_drop(0, nodes=2)
    tris = scx.surface_triangles(sc.tets, sc.rest)
    assert scx.detect_self(sc.rest, sc.rest, tris, margin=0.01) == []


@pytest.mark.parametrize("case", ["cube5", "star"])
def test_meshes_at_rest_have_no_self_contacts(case):
    """At rest no vertex faces another part of the surface within the margin.  The 5^3-node
    cube has vertices one layer from every convex edge, whose projections fall on the
    perpendicular face a voxel below its plane (excluded as not facing it and deeper than
    the margin); a star-profile mesh (the teaser's shape, fewer nodes) adds concave
    corners between its arms, thin walls and staircase steps."""
    if case == "cube5":
        sc = scenes.cube_drop(0)
        rest, tets, margin = sc.rest, sc.tets, sc.margin
    else:
        rest, tets = scenes.star_profile_mesh(0, target=(2000, 2400), layers=6)[:2]
        margin = 0.25 * 0.01
    tris = scx.surface_triangles(tets, rest)
    assert len(tris) > 100
    assert scx.detect_self(rest, rest, tris, margin=margin) == []


def test_facing_rule():
    """A vertex just outside a face but next to it across a convex edge (its own surface
    normal perpendicular to the face's) is not a contact; the same point on a separate body
    whose surface faces the face is."""
    tris = scx.surface_triangles(STACK_TETS, STACK)
    vn = scx.vertex_normals(STACK, tris)
    t = int(np.flatnonzero([sorted(tr) == [0, 1, 2] for tr in tris])[0])
    n, _ = scx.triangle_frame(*STACK[tris[t]])
    assert vn[4] @ n < 0.0  # the hovering vertex faces the bottom tet's top face
    X = STACK.copy()
    X[4:] += [0.0, 0.0, 0.001]
    X[4] = [0.2, 0.2, 0.003]
    assert (4, t) in scx.detect_self(X, X, tris, margin=0.01)
    # turn the top tet a quarter turn about vertex 4 (y axis): vertex 4's surface normal
    # becomes horizontal, perpendicular to the face it still hovers over
    Y = STACK.copy()
    Y[5:] = Y[4] + (STACK[5:] - STACK[4])[:, [2, 1, 0]] * [1.0, 1.0, -1.0]
    vy = scx.vertex_normals(Y, tris)
    assert abs(vy[4] @ n) <= 1e-15 and abs(vy[4][0]) > 0.1
    assert (4, t) not in scx.detect_self(Y, Y, tris, margin=0.01)


def test_hand_placed_contact():
    tris = scx.surface_triangles(STACK_TETS, STACK)
    pairs = scx.detect_self(STACK, STACK, tris, margin=0.01)
    assert len(pairs) == 1 and pairs[0][0] == 4
    assert sorted(tris[pairs[0][1]]) == [0, 1, 2]
    rows = scx.SelfRows(pairs, tris, STACK)
    # the weights reproduce the foot point (0.2, 0.2, 0); the gap is the hover height
    p = -(rows.signs[0, 1:, None] * STACK[rows.nodes[0, 1:]]).sum(0)
    np.testing.assert_allclose(p, [0.2, 0.2, 0.0], atol=1e-15)
    assert rows.gap[0] == pytest.approx(0.005)
    np.testing.assert_allclose(rows.C[0, 0], [0.0, 0.0, 1.0], atol=1e-15)
    # beyond the margin, or inside the body by more than the margin: no contact
    far = STACK.copy()
    far[4, 2] = 0.02
    assert scx.detect_self(far, far, tris, margin=0.01) == []
    deep = STACK.copy()
    deep[4, 2] = -0.011  # further inside than the margin
    assert scx.detect_self(deep, deep, tris, margin=0.01) == []
    # approaching: out of the margin at x_t, inside it at the predicted state
    pred = far.copy()
    pred[4, 2] = 0.004
    assert scx.detect_self(far, pred, tris, margin=0.01) == [(4, pairs[0][1])]


def test_contact_pair_forces_balance():
    """Newton's third law for any impulse (the weights sum to one), and zero torque when
    the vertex lies on the triangle (its lever arm equals the foot point's)."""
    X = STACK.copy()
    X[4, 2] = 0.0
    tris = scx.surface_triangles(STACK_TETS, STACK)
    rows = scx.SelfRows([(4, int(np.flatnonzero([sorted(t) == [0, 1, 2] for t in tris])[0]))], tris, X)
    rng = np.random.default_rng(0)
    for _ in range(5):
        lam = rng.normal(size=(1, 3))
        f = rows.H_T(lam, len(X))
        np.testing.assert_allclose(f.sum(0), 0.0, atol=1e-14)
        np.testing.assert_allclose(np.cross(X, f).sum(0), 0.0, atol=1e-14)
        assert np.abs(f).max() > 0.1


def test_delassus_equals_dense_product():
    """K and W of multi-node rows against H (A_n (x) I3)^-1 H^T with a dense inverse, for an
    arbitrary SPD A_n and rows sharing nodes."""
    rng = np.random.default_rng(3)
    n = 8
    G = rng.normal(size=(n, n))
    A = G @ G.T + n * np.eye(n)
    tris = scx.surface_triangles(STACK_TETS, STACK)
    X = STACK.copy()
    pairs = scx.detect_self(X, X, tris, margin=0.01)
    # a second row on the same triangle, from the top tet's vertex 5 placed under the face
    X2 = X.copy()
    X2[5] = [0.1, 0.3, -0.002]
    t = pairs[0][1]
    rows = scx.SelfRows([pairs[0], (5, t)], tris, X2)
    K, W = rows.delassus(lambda B: np.linalg.solve(A, B), n)
    Hm = rows.H(n)
    W_dense = Hm @ np.kron(np.linalg.inv(A), np.eye(3)) @ Hm.T
    np.testing.assert_allclose(W, W_dense, rtol=1e-12, atol=1e-14)
    Ai = np.linalg.inv(A)
    for j in range(2):
        for k in range(2):
            ref = sum(rows.signs[j, a] * rows.signs[k, b] * Ai[rows.nodes[j, a], rows.nodes[k, b]]
                      for a in range(4) for b in range(4))
            assert K[j, k] == pytest.approx(ref, rel=1e-12)


def test_frictionless_self_contact_brute_force_and_momentum():
    """One frictionless self-contact in the affine frame problem y = a + h^2 W lambda
    (App. A): the brute-force NCP solution is the closed form -a_n / (h^2 K_jj); the
    corrected positions q = u + A^-1 h^2 H^T lambda close the linearised gap, and the
    correction carries no linear momentum (the pair's impulses cancel and the elastic
    part of A is translation invariant)."""
    from oracle import brute_ncp
    from oracle.sim import OracleSim
    tets = np.array([[0, 2, 1, 3], [4, 5, 6, 7]], np.int32)  # positively oriented
    sc = scenes.Scene("stack", STACK.copy(), tets, scenes.MODEL_COROT, 1e5, 0.3, 1000.0, 0.01,
                      np.zeros(3), [], 0.01, 1, 10, 1)
    o = OracleSim(sc)
    n, h = len(STACK), sc.h
    tris = scx.surface_triangles(tets, STACK)
    pairs = scx.detect_self(STACK, STACK, tris, margin=0.01)
    rows = scx.SelfRows(pairs, tris, STACK)
    K, W = rows.delassus(o.lu.solve, n)
    u = STACK.copy()
    u[4:, 2] -= 0.007  # the top tet moved down: vertex 4 ends 2 mm below the face
    a = (np.einsum("jab,jb->ja", rows.C, np.einsum("ja,jab->jb", rows.signs, u[rows.nodes]))).reshape(-1)
    assert a[0] == pytest.approx(-0.002, abs=1e-12)
    sols = brute_ncp.solve_all(a, h * h * W, np.zeros(1))
    assert len(sols) == 1
    lam = np.asarray(sols[0]).reshape(1, 3)
    assert lam[0, 0] == pytest.approx(0.002 / (h * h * K[0, 0]), rel=1e-9)
    np.testing.assert_allclose(lam[0, 1:], 0.0, atol=1e-12)
    q = u + o.lu.solve(h * h * rows.H_T(lam, n))
    gap = rows.C[0, 0] @ (rows.signs[0] @ q[rows.nodes[0]])
    assert gap == pytest.approx(0.0, abs=1e-12)
    p = (o.mass[:, None] * (q - u)).sum(0)
    assert np.abs(p).max() <= 1e-12 * o.mass.sum() * 0.002


@pytest.mark.parametrize("mu,mode", [(2.0, "stick"), (0.05, "slide")])
def test_frictional_self_contact_brute_force(mu, mode):
    """The top tet pushed 7 mm down and 3 mm sideways into the bottom one's face: the
    brute-force Signorini-Coulomb solution is unique, closes the gap, and either sticks
    (no relative tangential motion, impulse inside the cone) or slides (impulse on the cone
    boundary, opposing the relative motion); the pair's impulses leave linear momentum
    unchanged in both cases."""
    from oracle import brute_ncp
    from oracle.sim import OracleSim
    tets = np.array([[0, 2, 1, 3], [4, 5, 6, 7]], np.int32)
    sc = scenes.Scene("stack", STACK.copy(), tets, scenes.MODEL_COROT, 1e5, 0.3, 1000.0, 0.01,
                      np.zeros(3), [], 0.01, 1, 10, 1)
    o = OracleSim(sc)
    n, h = len(STACK), sc.h
    tris = scx.surface_triangles(tets, STACK)
    rows = scx.SelfRows(scx.detect_self(STACK, STACK, tris, margin=0.01), tris, STACK)
    K, W = rows.delassus(o.lu.solve, n)
    u = STACK.copy()
    u[4:, 2] -= 0.007
    u[4:, 0] += 0.003
    rel = lambda x: np.einsum("ja,jab->jb", rows.signs, x[rows.nodes])  # x_v - p(x)
    a = np.einsum("jab,jb->ja", rows.C, rel(u))
    a[:, 1:] = np.einsum("jab,jb->ja", rows.C[:, 1:], rel(u - STACK))  # h delta_dot_f at u
    a = a.reshape(-1)
    # impulses are O(400) here: the mode checks take an absolute 1e-8 (2e-11 relative),
    # which the sliding mode's root finder reaches from 36 starting angles
    sols = brute_ncp.solve_all(a, h * h * W, np.array([mu]), tol=1e-8, n_starts=36)
    assert len(sols) == 1
    lam = np.asarray(sols[0])
    y = a + h * h * W @ lam
    assert lam[0] > 0.0 and y[0] == pytest.approx(0.0, abs=1e-12)
    lf, yf = lam[1:], y[1:]
    if mode == "stick":
        np.testing.assert_allclose(yf, 0.0, atol=1e-12)
        assert np.linalg.norm(lf) < mu * lam[0]
    else:
        assert np.linalg.norm(yf) > 1e-6
        assert np.linalg.norm(lf) == pytest.approx(mu * lam[0], rel=1e-8)
        assert np.dot(lf, yf) == pytest.approx(-np.linalg.norm(lf) * np.linalg.norm(yf), rel=1e-6)
    q = u + o.lu.solve(h * h * rows.H_T(lam.reshape(1, 3), n))
    p = (o.mass[:, None] * (q - u)).sum(0)
    assert np.abs(p).max() <= 1e-12 * o.mass.sum() * 0.002


# ---------------------------------------------------------------- the frame loop with self rows
def _fork_run(mu, frames=14, iters=0):
    from oracle.sim import OracleSim
    sc = scenes.fork_clap(0, mu=mu)
    o = OracleSim(sc)
    p0 = (o.mass[:, None] * o.v).sum(0)
    stats, gaps = [], []
    for _ in range(frames):
        q_t, q_pred, fc, lam = o.begin_frame()
        q = q_pred.copy()
        k = 0
        while True:
            q, lam, _ = o.iterate(fc, q, lam, q_t, q_pred, o.t + o.h, cr="exact")
            k += 1
            res = o.residual(fc, q, q_t, lam)
            if (iters and k >= iters) or (not iters and (res <= 1e-6 or k >= 60)):
                break
        if fc.c:
            gaps.append((res, np.einsum("ji,ji->j", fc.C[:, 0, :], fc.rows(q)) - fc.d_n, lam[:, 0].copy()))
        o.end_frame(q_t, q, fc, lam)
        stats.append((fc.c, k, res, np.abs((o.mass[:, None] * o.v).sum(0) - p0).max()))
    return o, stats, gaps


@pytest.mark.parametrize("mu", [0.0, 0.4])
def test_self_contact_frames_conserve_momentum(mu):
    """With no gravity, pins or obstacles, every force is internal: the elastic terms sum to
    zero over a tet, and a self-contact row's impulse acts as +C^T lambda on the vertex and
    -w_a C^T lambda on the triangle's corners with sum w_a = 1.  The fork's prongs collide
    over several frames; linear momentum stays at its initial value (zero) to rounding,
    at a fixed iteration count (5) as at convergence."""
    for iters in (5, 0):
        o, stats, _ = _fork_run(mu, iters=iters)
        assert max(c for c, *_ in stats) >= 4
        scale = o.mass.sum() * 0.6
        assert max(d for *_, d in stats) <= 1e-12 * scale, stats


def test_self_contact_frames_do_not_penetrate():
    """Frictionless fork: at every frame whose iteration reached NCP residual 1e-6 m, each
    self-contact row's gap is above -1e-6 m, and rows with a positive normal impulse are
    closed to 1e-6 m (the Signorini conditions of the vertex-triangle rows)."""
    _, stats, gaps = _fork_run(0.0)
    checked = 0
    for res, gap, lam_n in gaps:
        if res > 1e-6:
            continue
        checked += 1
        assert gap.min() >= -1e-6
        assert np.all(np.abs(gap[lam_n > 0]) <= 1e-6)
    assert checked >= 3
