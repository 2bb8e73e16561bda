"""Pins of the FP64 oracle against what the method and the mathematics fix.

Each test names the property it pins and the part of the method it guards:
exactness of the CG2 strain on quadratic fields, zero strain under rigid
motion, symmetric stress, lumped-mass sums, the uniform-ice fixed point, the
yield ellipse, the frozen-velocity relaxation closed form, the adjointness of
strain and divergence, and the velocity update's fixed point (free drift).
"""
import numpy as np
import pytest

from synth_inputs import make_domain, perturbed_vertices, uniform_vertices


def parallelogram_vertices(nx, ny, hx, hy, shear):
    iy, ix = np.meshgrid(np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    X = ix * hx + iy * shear
    Y = iy * hy
    return np.stack([X.ravel(), Y.ravel()]).astype(np.float64)


def node_xy_affine(nx, ny, hx, hy, shear):
    iy, ix = np.meshgrid(np.arange(2 * ny + 1), np.arange(2 * nx + 1), indexing="ij")
    return (ix * hx / 2 + iy * shear / 2).ravel(), (iy * hy / 2).ravel()


def shoelace_areas(V, nx, ny):
    X = V[0].reshape(ny + 1, nx + 1)
    Y = V[1].reshape(ny + 1, nx + 1)
    # counter-clockwise: (0,0) (1,0) (1,1) (0,1)
    xs = [X[:-1, :-1], X[:-1, 1:], X[1:, 1:], X[1:, :-1]]
    ys = [Y[:-1, :-1], Y[:-1, 1:], Y[1:, 1:], Y[1:, :-1]]
    a = 0.0
    for i in range(4):
        a = a + xs[i] * ys[(i + 1) % 4] - xs[(i + 1) % 4] * ys[i]
    return (0.5 * a).ravel()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# --------------------------------------------------------------------------- P1
@pytest.mark.parametrize("ns", [3, 6, 8])
def test_cg2_strain_exact_for_quadratic_velocity(oracle_mod, ns):
    O = oracle_mod
    nx, ny, hx, hy, sh = 5, 4, 1200.0, 900.0, 250.0
    m = O.Mesh(nx, ny, ns, 1, parallelogram_vertices(nx, ny, hx, hy, sh))
    x, y = node_xy_affine(nx, ny, hx, hy, sh)
    xs, ys = x / 1e3, y / 1e3  # km, to keep the polynomial well scaled
    vx = 0.3 + 0.02 * xs - 0.05 * ys + 0.004 * xs ** 2 - 0.003 * xs * ys + 0.002 * ys ** 2
    vy = -0.1 + 0.01 * xs + 0.03 * ys - 0.001 * xs ** 2 + 0.005 * xs * ys - 0.004 * ys ** 2
    E = m.strain(np.stack([vx, vy]))
    # analytic strain rates (per metre), linear in x, y
    def eps(xq, yq):
        xk, yk = xq / 1e3, yq / 1e3
        dvxdx = (0.02 + 0.008 * xk - 0.003 * yk) / 1e3
        dvxdy = (-0.05 - 0.003 * xk + 0.004 * yk) / 1e3
        dvydx = (0.01 - 0.002 * xk + 0.005 * yk) / 1e3
        dvydy = (0.03 + 0.005 * xk - 0.008 * yk) / 1e3
        return np.array([dvxdx, 0.5 * (dvxdy + dvydx), dvydy])
    # DG coefficients: value at the cell centre, then the slopes along xi and eta
    ex, ey = np.meshgrid(np.arange(nx), np.arange(ny))
    ex, ey = ex.ravel(), ey.ravel()
    xc = ex * hx + ey * sh + 0.5 * hx + 0.5 * sh
    yc = ey * hy + 0.5 * hy
    c0 = eps(xc, yc)
    cxi = eps(xc + hx, yc) - c0          # d/dxi of a linear function = change over one hx
    ceta = eps(xc + sh, yc + hy) - c0
    scale = np.abs(c0).max()
    for c in range(3):
        assert np.abs(E[c, 0] - c0[c]).max() < 1e-13 * scale
        assert np.abs(E[c, 1] - cxi[c]).max() < 1e-13 * scale
        assert np.abs(E[c, 2] - ceta[c]).max() < 1e-13 * scale
        for k in range(3, ns):
            assert np.abs(E[c, k]).max() < 1e-13 * scale


# --------------------------------------------------------------------------- P2
@pytest.mark.parametrize("ns", [3, 6])
def test_rigid_motion_gives_zero_strain(oracle_mod, ns):
    O = oracle_mod
    nx, ny = 6, 5
    V = perturbed_vertices(nx, ny, 2000.0, 2000.0, amp=0.15, seed=3)
    m = O.Mesh(nx, ny, ns, 1, V)
    # CG2 node positions of a bilinear mesh are the images of the reference nodes;
    # a translation does not need them
    v = np.stack([np.full(m.nn, 0.7), np.full(m.nn, -0.2)])
    E = m.strain(v)
    assert np.abs(E).max() < 1e-18
    # rotation on an affine mesh (node positions known in closed form)
    hx, hy, sh = 1500.0, 1000.0, 300.0
    m2 = O.Mesh(nx, ny, ns, 1, parallelogram_vertices(nx, ny, hx, hy, sh))
    x, y = node_xy_affine(nx, ny, hx, hy, sh)
    om = 1e-5
    E2 = m2.strain(np.stack([-om * y, om * x]))
    assert np.abs(E2).max() < 1e-13 * om


# --------------------------------------------------------------------------- P3
def test_rotation_leaves_isotropic_pressure_and_shear_rows_use_s12(oracle_mod):
    O = oracle_mod
    p = O.Params()
    nx, ny, hx, hy, sh = 4, 3, 1500.0, 1000.0, 200.0
    m = O.Mesh(nx, ny, 6, 1, parallelogram_vertices(nx, ny, hx, hy, sh))
    x, y = node_xy_affine(nx, ny, hx, hy, sh)
    E = m.strain(np.stack([-2e-6 * y, 2e-6 * x]))
    H = np.full((1, m.ne), 1.4)
    A = np.full((1, m.ne), 0.9)
    S = m.stress(p, E, H, A, np.zeros((3, 6, m.ne)))
    P = p.Pstar * 1.4 * np.exp(-p.C * 0.1)
    np.testing.assert_allclose(S[0, 0], -0.5 * P / p.alpha, rtol=1e-10)
    np.testing.assert_allclose(S[2, 0], -0.5 * P / p.alpha, rtol=1e-10)
    assert np.abs(S[1]).max() < 1e-10 * P
    assert np.abs(S[0, 1:]).max() < 1e-10 * P
    # a uniform pure shear stress on one rectangle: F_x = -s12 int dphi/dy, F_y = -s12 int dphi/dx
    m1 = O.Mesh(1, 1, 6, 1, uniform_vertices(1, 1, 3.0, 2.0))
    S1 = np.zeros((3, 6, 1))
    S1[1, 0, 0] = 5.0
    F = m1.divergence(S1)
    w = np.array([1 / 6, 2 / 3, 1 / 6])
    jump = np.array([-1.0, 0.0, 1.0])  # L_c(1) - L_c(0)
    for a in range(9):
        b, c = a // 3, a % 3
        j = b * 3 + c  # 3x3 nodes of a 1x1 mesh
        int_dx = 2.0 * jump[c] * w[b]   # hy * (L_c(1)-L_c(0)) * int L_b
        int_dy = 3.0 * w[c] * jump[b]   # hx * int L_c * (L_b(1)-L_b(0))
        assert abs(F[0, j] - (-5.0 * int_dy)) < 1e-13
        assert abs(F[1, j] - (-5.0 * int_dx)) < 1e-13


# --------------------------------------------------------------------------- P4
@pytest.mark.parametrize("ns", [3, 6])
def test_lumped_mass_sums_equal_integrals(oracle_mod, ns):
    O = oracle_mod
    p = O.Params()
    nx, ny = 7, 5
    V = perturbed_vertices(nx, ny, 800.0, 800.0, amp=0.2, seed=11)
    m = O.Mesh(nx, ny, ns, 1, V)
    rng = np.random.default_rng(1)
    H = rng.uniform(0.5, 2.0, (1, m.ne))
    A = rng.uniform(0.7, 1.3, (1, m.ne))  # some above 1: clamped to 1
    MH, mA = m.node_masses(p, H, A)
    area = shoelace_areas(V, nx, ny)
    assert rel(MH.sum(), p.rho_i * np.dot(H[0], area)) < 1e-13
    assert rel(mA.sum(), np.dot(np.minimum(A[0], 1.0), area)) < 1e-13
    assert (MH > 0).all() and (mA > 0).all()


def test_lumped_mass_per_node_weights_uniform_mesh(oracle_mod):
    O = oracle_mod
    p = O.Params()
    nx, ny, h = 4, 3, 1000.0
    m = O.Mesh(nx, ny, 6, 1, uniform_vertices(nx, ny, h))
    MH, mA = m.node_masses(p, np.full((1, m.ne), 2.0), np.full((1, m.ne), 1.0))
    NX = 2 * nx + 1
    area = h * h
    def at(ix, iy):
        return mA[iy * NX + ix]
    assert abs(at(0, 0) - area / 36) < 1e-9                 # domain corner
    assert abs(at(2, 0) - 2 * area / 36) < 1e-9             # boundary vertex
    assert abs(at(2, 2) - 4 * area / 36) < 1e-9             # interior vertex
    assert abs(at(1, 2) - 2 * area / 9) < 1e-9              # interior edge midpoint
    assert abs(at(1, 1) - 4 * area / 9) < 1e-9              # element centre
    np.testing.assert_allclose(MH, p.rho_i * 2.0 * mA, rtol=1e-14)


# --------------------------------------------------------------------------- P5
@pytest.mark.parametrize("ns,perturb", [(3, 0.0), (6, 0.0), (6, 0.15)])
def test_uniform_ice_rest_state_is_fixed_point(oracle_mod, ns, perturb):
    O = oracle_mod
    p = O.Params()
    d = make_domain(6, 5, ns, 1, seed=4, h=2000.0, perturb=perturb)
    m = O.Mesh(d.nx, d.ny, ns, 1, d.vertices)
    H = np.full((1, m.ne), 1.2)
    A = np.full((1, m.ne), 0.95)
    P = p.Pstar * 1.2 * np.exp(-p.C * 0.05)
    S0 = np.zeros((3, ns, m.ne))
    S0[0, 0] = -0.5 * P
    S0[2, 0] = -0.5 * P
    z = np.zeros((2, m.nn))
    # one subcycle: only rounding moves the state. A wrong sign or a broken partition of
    # unity would give |v| ~ P h / (M^H (1+beta) / dt) ~ 1 m/s and S changes of order P.
    v, S = m.step(p, H, A, z, z, z, S0, 1)
    assert np.abs(v).max() < 1e-13
    assert rel(S, S0) < 1e-14
    # five subcycles: the rounding-size velocity is seen through the viscous stiffness
    # P / Delta_min ~ 1e13 1/s, so the bound is looser but still far below order one
    v, S = m.step(p, H, A, z, z, z, S0, 5)
    assert np.abs(v).max() < 1e-10
    assert rel(S, S0) < 1e-9


# --------------------------------------------------------------------------- P7
def test_stress_on_yield_ellipse(oracle_mod):
    O = oracle_mod
    p = O.Params()
    d = make_domain(4, 4, 6, 3, seed=9, h=1000.0, perturb=0.1, ho_amp=0.3)
    m = O.Mesh(4, 4, 6, 3, d.vertices)
    rng = np.random.default_rng(2)
    # strain rates from tiny (viscous regime) to large (plastic regime)
    E = rng.normal(0, 1, (3, 6, m.ne)) * 10.0 ** rng.uniform(-11, -5, (1, 1, m.ne))
    s, P, D = m.stress_gauss(p, E, d.H, d.A)
    sI = 0.5 * (s[0] + s[2])
    sII = np.sqrt((0.5 * (s[0] - s[2])) ** 2 + s[1] ** 2)
    ok = P > 0
    assert ok.sum() > 10
    lhs = ((sI[ok] + P[ok] / 2) / (P[ok] / 2)) ** 2 + (sII[ok] / (P[ok] / 4)) ** 2
    rhs = 1.0 - p.DeltaMin ** 2 / D[ok] ** 2
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)
    # where the clamped thickness is zero there is no stress at all
    assert (np.abs(s[:, ~ok]) == 0).all()


# --------------------------------------------------------------------------- P13
def test_listing_constants_are_hibler_ellipse_e2(oracle_mod):
    """Eq. (si:mevp): sigma_vp = eta (grad v + grad v^T) + zeta div v I - P/2 I with
    Hibler's zeta = P/(2 Delta), eta = zeta/e^2 and e = 2."""
    O = oracle_mod
    p = O.Params()
    d = make_domain(3, 3, 6, 1, seed=21, h=1000.0)
    m = O.Mesh(3, 3, 6, 1, d.vertices)
    rng = np.random.default_rng(4)
    E = rng.normal(0, 1e-7, (3, 6, m.ne))
    s, P, D = m.stress_gauss(p, E, d.H, d.A)
    e11, e12, e22 = m.eval_gauss(E)
    ecc = 2.0
    Dh = np.sqrt(p.DeltaMin ** 2 + (e11 ** 2 + e22 ** 2) * (1 + ecc ** -2) + 4 * ecc ** -2 * e12 ** 2
                 + 2 * e11 * e22 * (1 - ecc ** -2))
    zeta = P / (2 * Dh)
    eta = zeta / ecc ** 2
    div = e11 + e22
    np.testing.assert_allclose(D, Dh, rtol=1e-14)
    np.testing.assert_allclose(s[0], 2 * eta * e11 + (zeta - eta) * div - P / 2, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(s[1], 2 * eta * e12, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(s[2], 2 * eta * e22 + (zeta - eta) * div - P / 2, rtol=1e-12, atol=1e-9)


def test_ice_clamps(oracle_mod):
    """h = max(0, H Psi), a = min(1, max(0, A Psi)) (both stress listings)."""
    O = oracle_mod
    p = O.Params()
    m = O.Mesh(2, 1, 6, 3, uniform_vertices(2, 1, 1000.0))
    H = np.array([[0.1, 1.0], [2.0, 0.0], [0.0, 0.0]])   # element 0: h < 0 at xi < 0.45
    A = np.array([[0.99, 1.05], [0.5, 0.0], [0.0, 0.0]])  # element 1: a > 1 everywhere
    E = np.zeros((3, 6, 2))
    s, P, D = m.stress_gauss(p, E, H, A)
    gp = oracle_mod.tables(6)[0]
    xi = np.tile(gp, 3)
    h0 = 0.1 + 2.0 * (xi - 0.5)
    a0 = np.clip(0.99 + 0.5 * (xi - 0.5), 0.0, 1.0)
    np.testing.assert_allclose(P[:, 0], p.Pstar * np.maximum(h0, 0) * np.exp(-p.C * (1 - a0)), rtol=1e-14)
    assert (P[h0 < 0, 0] == 0).all()
    np.testing.assert_allclose(P[:, 1], p.Pstar * 1.0, rtol=1e-15)


# --------------------------------------------------------------------------- P8
@pytest.mark.parametrize("relax_form", [0, 1])
def test_frozen_velocity_relaxation_closed_form(oracle_mod, relax_form):
    O = oracle_mod
    p = O.Params(relax_form=relax_form, alpha=7.0)
    d = make_domain(3, 4, 6, 1, seed=5, h=1500.0, perturb=0.1)
    m = O.Mesh(3, 4, 6, 1, d.vertices)
    rng = np.random.default_rng(8)
    E = rng.normal(0, 1e-6, (3, 6, m.ne))
    S0 = rng.normal(0, 1e3, (3, 6, m.ne))
    target = m.stress(O.Params(relax_form=0, alpha=1.0), E, d.H, d.A, S0)  # alpha = 1: S = Pi(s)
    fac = 1 - 1 / p.alpha if relax_form == 0 else p.alpha / (1 + p.alpha)
    S = S0
    for k in range(1, 13):
        S = m.stress(p, E, d.H, d.A, S)
        if relax_form == 0:
            expect = fac ** k * S0 + (1 - fac ** k) * target
        else:
            # alpha/(1+alpha) and 1/(1+alpha) sum to one as well
            expect = fac ** k * S0 + (1 - fac ** k) * target
        assert rel(S, expect) < 1e-12


# --------------------------------------------------------------------------- P9
@pytest.mark.parametrize("ns", [3, 6])
def test_divergence_is_adjoint_of_strain(oracle_mod, ns):
    O = oracle_mod
    d = make_domain(5, 4, ns, 1, seed=6, h=1000.0, perturb=0.15)
    m = O.Mesh(5, 4, ns, 1, d.vertices)
    rng = np.random.default_rng(3)
    S = rng.normal(0, 1e3, (3, ns, m.ne))
    w = rng.normal(0, 1.0, (2, m.nn))
    F = m.divergence(S)
    lhs = np.sum(F * w)
    eps = m.strain_gauss(w)                      # [3][nG][ne]
    sig = m.eval_gauss(S)                        # [3][nG][ne]
    wdet = np.stack([m.element_geometry(e)[0] for e in range(m.ne)], axis=1)  # [nG][ne]
    # sigma : eps(w) with the off-diagonal counted twice
    rhs = -np.sum(wdet * (sig[0] * eps[0] + 2 * sig[1] * eps[1] + sig[2] * eps[2]))
    assert abs(lhs - rhs) < 1e-12 * np.sum(np.abs(F * w))


# --------------------------------------------------------------------------- P10
def test_velocity_update_without_forces_relaxes_toward_vn(oracle_mod):
    O = oracle_mod
    p = O.Params(C_a=0.0, C_o=0.0, f_cor=0.0, beta=5.0)
    m = O.Mesh(3, 3, 6, 1, uniform_vertices(3, 3, 1000.0))
    rng = np.random.default_rng(0)
    MH, mA = m.node_masses(p, np.full((1, m.ne), 1.0), np.full((1, m.ne), 0.9))
    vprev = rng.normal(0, 0.1, (2, m.nn))
    vn = rng.normal(0, 0.1, (2, m.nn))
    v = m.velocity(p, np.zeros((2, m.nn)), MH, mA, np.zeros((2, m.nn)), np.zeros((2, m.nn)), vn, vprev)
    NX = 2 * 3 + 1
    ix, iy = np.arange(m.nn) % NX, np.arange(m.nn) // NX
    interior = (ix > 0) & (iy > 0) & (ix < NX - 1) & (iy < NX - 1)
    np.testing.assert_allclose(v[:, interior], (p.beta * vprev + vn)[:, interior] / (1 + p.beta), rtol=1e-14)
    assert (v[:, ~interior] == 0).all()


def test_mevp_fixed_point_solves_implicit_free_drift(oracle_mod):
    """With no internal stress (P* = 0) the pseudo-time iteration must converge to the
    backward-Euler momentum balance of Eq. (si:momentum): rho H (v - v^n)/dt = tau_a + tau_o(v)
    - rho H f k x v, node by node with lumped masses."""
    O = oracle_mod
    p = O.Params(Pstar=0.0, beta=2.0)
    d = make_domain(4, 4, 6, 1, seed=12, h=5000.0)
    m = O.Mesh(4, 4, 6, 1, d.vertices)
    rng = np.random.default_rng(7)
    vn = rng.normal(0, 0.05, (2, m.nn))
    v, S = m.subcycles(p, d.H, d.A, d.wind, d.ocean, vn, vn.copy(), np.zeros((3, 6, m.ne)), 200)
    assert np.abs(S).max() == 0.0
    MH, mA = m.node_masses(p, d.H, d.A)
    tau = p.rho_a * p.C_a * np.hypot(d.wind[0], d.wind[1]) * d.wind
    rel_o = d.ocean - v
    tau_o = p.rho_o * p.C_o * np.hypot(rel_o[0], rel_o[1]) * rel_o
    kxv = np.stack([-v[1], v[0]])
    res = MH / p.dt * (v - vn) - mA * tau - mA * tau_o + p.f_cor * MH * kxv
    NX = 9
    ix, iy = np.arange(m.nn) % NX, np.arange(m.nn) // NX
    interior = (ix > 0) & (iy > 0) & (ix < NX - 1) & (iy < NX - 1)
    scale = np.abs(mA * tau).max()
    assert np.abs(res[:, interior]).max() < 1e-10 * scale
    assert np.abs(v).max() > 1e-3  # the wind actually moved the ice


# --------------------------------------------------------------------------- misc
def test_full_step_is_deterministic_and_thread_independent(oracle_mod):
    O = oracle_mod
    p = O.Params()
    d = make_domain(12, 10, 6, 1, seed=13, h=4000.0, perturb=0.1)
    m = O.Mesh(12, 10, 6, 1, d.vertices)
    v1, S1 = m.run(p, d.H, d.A, d.wind, d.ocean, 2, 20)
    v2, S2 = m.run(p, d.H, d.A, d.wind, d.ocean, 2, 20)
    assert np.array_equal(v1, v2) and np.array_equal(S1, S2)
    assert np.abs(v1).max() > 0 and np.isfinite(S1).all()


def test_mesh_validation(oracle_mod):
    O = oracle_mod
    V = uniform_vertices(2, 2, 1.0)
    for ns, na in [(5, 1), (6, 2), (4, 3)]:
        with pytest.raises(ValueError):
            O.Mesh(2, 2, ns, na, V)
    Vf = V.copy()
    Vf[0] = Vf[0][::-1].copy()  # mirrored -> negative Jacobians
    with pytest.raises(ValueError):
        O.Mesh(2, 2, 6, 1, Vf)


# --------------------------------------------------------------------------- projection
@pytest.mark.parametrize("ns", [3, 6, 8])
def test_projection_is_identity_on_dg_space_and_orthogonal(oracle_mod, ns):
    """Pi_e = M_e^-1 Psi W_e (the listings' iMJwPSI) on non-affine elements: it returns the
    coefficients of any function already in the DG space, and its residual is W_e-orthogonal
    to every DG basis function."""
    O = oracle_mod
    d = make_domain(5, 4, ns, 1, seed=31, h=1000.0, perturb=0.25)
    m = O.Mesh(5, 4, ns, 1, d.vertices)
    rng = np.random.default_rng(17)
    c = rng.normal(0, 1, (3, ns, m.ne))
    back = m.project(m.eval_gauss(c))
    assert rel(back, c) < 1e-13
    g = rng.normal(0, 1, (2, m.ng, m.ne))
    res = g - m.eval_gauss(m.project(g))
    psiS = O.tables(ns)[2]
    wdet = np.stack([m.element_geometry(e)[0] for e in range(m.ne)], axis=1)
    inner = np.einsum("kq,qe,cqe->cke", psiS, wdet, res)
    assert np.abs(inner).max() < 1e-12 * np.abs(np.einsum("kq,qe,cqe->cke", psiS, wdet, g)).max()


def test_oracle_result_does_not_depend_on_its_thread_count():
    """Every parallel loop of the oracle writes disjoint outputs and sums in a
    fixed order, so one thread and all threads give the same bits."""
    import oracle
    from synth_inputs import make_domain
    d = make_domain(16, 12, 6, 1, seed=8, h=10e3, perturb=0.1)
    m = oracle.Mesh(d.nx, d.ny, d.n_s, d.n_a, d.vertices)
    p = oracle.Params()
    many = m.run(p, d.H, d.A, d.wind, d.ocean, 2, 10)
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        one = m.run(p, d.H, d.A, d.wind, d.ocean, 2, 10)
    finally:
        oracle.set_num_threads(threads)
    assert all(np.array_equal(a, b) for a, b in zip(many, one))
