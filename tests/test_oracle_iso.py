"""Pins of the oracle's isoparametric geometry (reading R8: the cell map in the
velocity's CG2 space, Sec. 2.1, so cells may have curved edges).

* On a bilinear mesh whose CG2 nodes are placed by the bilinear map, the
  isoparametric oracle equals the bilinear (already pinned) oracle.
* On curved meshes: a velocity linear in the physical coordinates is in the
  isoparametric space, so its strain is the exact constant; cell areas
  (sum of w |J|) equal Green's theorem on the four quadratic edges (Simpson's
  rule, exact for the cubic integrand); lumped masses sum to rho_i H area;
  the divergence is the adjoint of the strain; the projection is the identity
  on the DG space; advection conserves mass and keeps a constant constant
  under a rotation.
"""
import numpy as np
import pytest

from synth_inputs import curved_nodes, make_domain, perturbed_vertices


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def bilinear_nodes(V, nx, ny):
    """CG2 node positions of a bilinear mesh: corners, edge midpoints and cell
    centres are the images of the reference nodes under each cell's bilinear map."""
    X = V[0].reshape(ny + 1, nx + 1)
    Y = V[1].reshape(ny + 1, nx + 1)
    out = []
    for C in (X, Y):
        N = np.zeros((2 * ny + 1, 2 * nx + 1))
        N[::2, ::2] = C
        N[::2, 1::2] = 0.5 * (C[:, :-1] + C[:, 1:])
        N[1::2, ::2] = 0.5 * (C[:-1, :] + C[1:, :])
        N[1::2, 1::2] = 0.25 * (C[:-1, :-1] + C[:-1, 1:] + C[1:, :-1] + C[1:, 1:])
        out.append(N.ravel())
    return np.stack(out)


def green_areas(nodes, nx, ny):
    """Area of every cell from its 4 quadratic edges: A = 1/2 sum over the
    counter-clockwise edges of int (x y' - y x') du, Simpson's rule (exact:
    the integrand is cubic in the edge parameter)."""
    NX = 2 * nx + 1
    X = nodes[0].reshape(2 * ny + 1, NX)
    Y = nodes[1].reshape(2 * ny + 1, NX)
    areas = np.zeros(nx * ny)
    for ey in range(ny):
        for ex in range(nx):
            i0, j0 = 2 * ey, 2 * ex
            # edges as (start, middle, end) node (row, col), counter-clockwise
            edges = [((i0, j0), (i0, j0 + 1), (i0, j0 + 2)),
                     ((i0, j0 + 2), (i0 + 1, j0 + 2), (i0 + 2, j0 + 2)),
                     ((i0 + 2, j0 + 2), (i0 + 2, j0 + 1), (i0 + 2, j0)),
                     ((i0 + 2, j0), (i0 + 1, j0), (i0, j0))]
            a = 0.0
            for p0, pm, p1 in edges:
                xs = np.array([X[p0], X[pm], X[p1]])
                ys = np.array([Y[p0], Y[pm], Y[p1]])
                f = 0.0
                for u, wt in ((0.0, 1 / 6), (0.5, 4 / 6), (1.0, 1 / 6)):
                    L = np.array([(1 - u) * (1 - 2 * u), 4 * u * (1 - u), u * (2 * u - 1)])
                    dL = np.array([4 * u - 3, 4 - 8 * u, 4 * u - 1])
                    x, y = L @ xs, L @ ys
                    xp, yp = dL @ xs, dL @ ys
                    f += wt * (x * yp - y * xp)
                a += 0.5 * f
            areas[ey * nx + ex] = a
    return areas


def curved_mesh(oracle_mod, nx, ny, ns, na, h=2000.0, amp=0.15, seed=5):
    nodes = curved_nodes(nx, ny, h, h, amp=amp, seed=seed)
    return oracle_mod.Mesh(nx, ny, ns, na, nodes=nodes), nodes


@pytest.mark.parametrize("ns", [3, 6])
def test_iso_map_of_bilinear_nodes_equals_bilinear_mesh(oracle_mod, ns):
    O = oracle_mod
    nx, ny = 12, 10
    d = make_domain(nx, ny, ns, 1, seed=21, h=10e3, perturb=0.15)
    mb = O.Mesh(nx, ny, ns, 1, d.vertices)
    mi = O.Mesh(nx, ny, ns, 1, nodes=bilinear_nodes(d.vertices, nx, ny))
    for e in (0, 37, nx * ny - 1):
        for a, b in zip(mi.element_geometry(e), mb.element_geometry(e)):
            assert rel(a, b) < 1e-13
    p = O.Params()
    vb, Sb = mb.run(p, d.H, d.A, d.wind, d.ocean, 2, 20)
    vi, Si = mi.run(p, d.H, d.A, d.wind, d.ocean, 2, 20)
    assert np.abs(vb).max() > 1e-4
    assert rel(vi, vb) < 1e-12 and rel(Si, Sb) < 1e-12
    rng = np.random.default_rng(2)
    NX = 2 * nx + 1
    ix, iy = np.arange(mb.nn) % NX, np.arange(mb.nn) // NX
    inner = (ix > 0) & (iy > 0) & (ix < NX - 1) & (iy < 2 * ny)
    v = rng.normal(0, 0.2, (2, mb.nn)) * inner
    assert rel(mi.advect_rate(v, d.H), mb.advect_rate(v, d.H)) < 1e-12


@pytest.mark.parametrize("ns", [3, 6, 8])
def test_iso_linear_velocity_has_exact_constant_strain(oracle_mod, ns):
    """v = a + B x is in the isoparametric CG2 space (x itself is), so on curved
    cells its strain is sym(B) exactly: coefficient 0 = sym(B), the rest 0."""
    m, nodes = curved_mesh(oracle_mod, 6, 5, ns, 1)
    B = np.array([[2e-6, -3e-6], [5e-6, -1e-6]])
    a = np.array([0.3, -0.1])
    v = a[:, None] + B @ nodes
    E = m.strain(v)
    want = [B[0, 0], 0.5 * (B[0, 1] + B[1, 0]), B[1, 1]]
    scale = np.abs(B).max()
    for c in range(3):
        assert np.abs(E[c, 0] - want[c]).max() < 1e-12 * scale
        assert np.abs(E[c, 1:]).max() < 1e-12 * scale


@pytest.mark.parametrize("ns", [3, 6])
def test_iso_cell_areas_and_lumped_mass_match_greens_theorem(oracle_mod, ns):
    nx, ny = 7, 6
    m, nodes = curved_mesh(oracle_mod, nx, ny, ns, 1, seed=8)
    areas = green_areas(nodes, nx, ny)
    wsum = np.array([m.element_geometry(e)[0].sum() for e in range(m.ne)])
    assert rel(wsum, areas) < 1e-13
    # the mesh is genuinely curved: the straight-edge (shoelace) areas differ
    NX = 2 * nx + 1
    corner = (np.arange(ny + 1)[:, None] * 2 * NX + np.arange(nx + 1)[None, :] * 2).ravel()
    V = nodes[:, corner]
    Xc = V[0].reshape(ny + 1, nx + 1)
    Yc = V[1].reshape(ny + 1, nx + 1)
    xs = [Xc[:-1, :-1], Xc[:-1, 1:], Xc[1:, 1:], Xc[1:, :-1]]
    ys = [Yc[:-1, :-1], Yc[:-1, 1:], Yc[1:, 1:], Yc[1:, :-1]]
    shoe = 0.5 * sum(xs[i] * ys[(i + 1) % 4] - xs[(i + 1) % 4] * ys[i] for i in range(4))
    assert rel(shoe.ravel(), areas) > 1e-4
    p = oracle_mod.Params()
    H = np.random.default_rng(4).uniform(0.5, 2.0, (1, m.ne))
    A = np.full((1, m.ne), 0.9)
    MH, mA = m.node_masses(p, H, A)
    assert abs(MH.sum() - p.rho_i * np.sum(H[0] * areas)) < 1e-12 * MH.sum()
    assert abs(mA.sum() - 0.9 * areas.sum()) < 1e-12 * mA.sum()


@pytest.mark.parametrize("ns", [3, 6])
def test_iso_divergence_is_adjoint_of_strain(oracle_mod, ns):
    m, _ = curved_mesh(oracle_mod, 5, 4, ns, 1, seed=6)
    rng = np.random.default_rng(3)
    S = rng.normal(0, 1e3, (3, ns, m.ne))
    w = rng.normal(0, 1.0, (2, m.nn))
    F = m.divergence(S)
    eps = m.strain_gauss(w)
    sig = m.eval_gauss(S)
    wdet = np.stack([m.element_geometry(e)[0] for e in range(m.ne)], axis=1)
    rhs = -np.sum(wdet * (sig[0] * eps[0] + 2 * sig[1] * eps[1] + sig[2] * eps[2]))
    assert abs(np.sum(F * w) - rhs) < 1e-12 * np.sum(np.abs(F * w))


@pytest.mark.parametrize("ns", [3, 6, 8])
def test_iso_projection_is_identity_on_dg_space(oracle_mod, ns):
    m, _ = curved_mesh(oracle_mod, 5, 4, ns, 1, seed=9)
    c = np.random.default_rng(17).normal(0, 1, (3, ns, m.ne))
    assert rel(m.project(m.eval_gauss(c)), c) < 1e-13


def test_iso_uniform_ice_rest_state_is_fixed_point(oracle_mod):
    """Uniform ice at rest with S = Pi(-P/2 I), no forcing: interior nodal forces
    vanish by the partition of unity on curved cells too."""
    O = oracle_mod
    nx, ny, ns = 6, 5, 6
    m, _ = curved_mesh(O, nx, ny, ns, 1, h=5e3, seed=11)
    p = O.Params()
    H = np.full((1, m.ne), 1.3)
    A = np.full((1, m.ne), 0.95)
    P = p.Pstar * 1.3 * np.exp(-p.C * (1 - 0.95))
    S = np.zeros((3, ns, m.ne))
    S[0, 0] = S[2, 0] = -P / 2
    z = np.zeros((2, m.nn))
    # bounds as for bilinear cells: a broken partition of unity or a wrong sign
    # would give |v| ~ 1 m/s and S changes of order P
    v, S1 = m.step(p, H, A, z, z, z, S, 1)
    assert np.abs(v).max() < 1e-13
    assert rel(S1, S) < 1e-14
    v, S1 = m.step(p, H, A, z, z, z, S, 5)
    assert np.abs(v).max() < 1e-10
    assert rel(S1, S) < 1e-9


def test_iso_advection_conserves_mass_and_keeps_constant_under_rotation(oracle_mod):
    O = oracle_mod
    nx, ny = 8, 7
    m, nodes = curved_mesh(O, nx, ny, 6, 1, h=2e3, seed=12)
    areas = green_areas(nodes, nx, ny)
    NX = 2 * nx + 1
    ix, iy = np.arange(m.nn) % NX, np.arange(m.nn) // NX
    inner = (ix > 0) & (iy > 0) & (ix < NX - 1) & (iy < 2 * ny)
    rng = np.random.default_rng(5)
    v = rng.normal(0, 0.3, (2, m.nn)) * inner
    H = rng.uniform(0.5, 2.0, (1, m.ne))
    A = rng.uniform(0.8, 1.0, (1, m.ne))
    H1, A1 = H, A
    for _ in range(3):
        H1, A1 = m.advect(600.0, v, H1, A1)
    assert np.abs(H1 - H).max() > 1e-4
    assert abs(np.sum(H1[0] * areas) - np.sum(H[0] * areas)) < 1e-12 * np.sum(H[0] * areas)
    # a rotation about an interior point is linear in x: in the isoparametric
    # space, divergence-free, and every integral of the rate is exact
    om = 2e-5
    x, y = nodes
    rot = np.stack([-om * (y - 6000.0), om * (x - 7000.0)])
    C = np.full((1, m.ne), 1.7)
    assert np.abs(m.advect_rate(rot, C)).max() < 1e-15


def test_iso_mesh_validation(oracle_mod):
    O = oracle_mod
    nodes = curved_nodes(4, 3, 1000.0, amp=0.1, seed=1)
    with pytest.raises(ValueError):
        O.Mesh(4, 3, 6, 1, nodes=nodes[:, :-1])
    bad = nodes.copy()
    NX = 9
    bad[0, 1 * NX + 1] += 2000.0  # fold a cell: non-positive Jacobian
    with pytest.raises(ValueError):
        O.Mesh(4, 3, 6, 1, nodes=bad)
    with pytest.raises(ValueError):
        O.Mesh(4, 3, 6, 1)


def test_iso_geometry_is_translation_invariant(oracle_mod):
    """The cell geometry does not depend on where the mesh sits: the same curved
    mesh of 64 m cells moved ~2000 km away gives the same w|J| and gradients.
    Node positions are on a 2^-10 m grid, so the moved mesh is represented
    exactly; a Jacobian summed from absolute positions would lose ~7 digits to
    cancellation, one from positions relative to a cell node loses none."""
    nodes = np.round(curved_nodes(6, 5, 64.0, 64.0, amp=0.15, seed=21) * 1024.0) / 1024.0
    far = nodes + np.array([[2.0 ** 21], [-(2.0 ** 20)]])
    assert np.array_equal(far - np.array([[2.0 ** 21], [-(2.0 ** 20)]]), nodes)
    m0 = oracle_mod.Mesh(6, 5, 6, 1, nodes=nodes)
    m1 = oracle_mod.Mesh(6, 5, 6, 1, nodes=far)
    for e in (0, 13, 29):
        for a, b in zip(m1.element_geometry(e), m0.element_geometry(e)):
            assert rel(a, b) < 1e-14


@pytest.mark.parametrize("ns", [3, 6])
@pytest.mark.parametrize("kind", ["bilinear", "curved"])
def test_basis_gradients_reproduce_the_coordinates(oracle_mod, ns, kind):
    """The coordinate functions lie in each cell's CG2 space (the bilinear map
    is biquadratic-representable, the isoparametric map is one by definition),
    so at every Gauss point of every element the gradient tables give
    sum_a grad phi_a = 0, sum_a x_a grad phi_a = (1, 0) and
    sum_a y_a grad phi_a = (0, 1), with x_a, y_a the element's nine node
    positions (local node a = 3 b + c at row 2 ey + b, column 2 ex + c)."""
    nx, ny = 5, 4
    if kind == "bilinear":
        V = perturbed_vertices(nx, ny, 2000.0, amp=0.2, seed=9)
        m = oracle_mod.Mesh(nx, ny, ns, 1, V)
        nodes = bilinear_nodes(V, nx, ny)
    else:
        m, nodes = curved_mesh(oracle_mod, nx, ny, ns, 1)
    NX = 2 * nx + 1
    for e in range(m.ne):
        ex, ey = e % nx, e // nx
        idx = [(2 * ey + a // 3) * NX + 2 * ex + a % 3 for a in range(9)]
        xa, ya = nodes[0][idx], nodes[1][idx]
        wd, gx, gy = m.element_geometry(e)
        assert gx.shape == (9, m.ng) and (wd > 0).all()
        h = 2000.0
        for G, want in ((gx, (1.0, 0.0)), (gy, (0.0, 1.0))):
            assert np.abs(G.sum(axis=0)).max() < 1e-12 / h
            assert np.abs(xa @ G - want[0]).max() < 1e-12
            assert np.abs(ya @ G - want[1]).max() < 1e-12
