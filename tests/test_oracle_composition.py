"""Pins of the oracle's subcycle composition and of the routing inside its
stress and velocity updates.

The per-phase pins (strain exactness, yield ellipse, adjointness, masses) fix
each phase on inputs where a component mix-up or a wrong sign in the glue
between phases would not show. These tests close that gap:

* the velocity update returns the solution of the lumped momentum balance it
  is defined by (the semi-discrete Eq. (si:momentum) under the pseudo-time
  relaxation of Eq. (si:mevp)), with a non-zero nodal force, drag and Coriolis;
* the stress update of every component and every DG coefficient equals the
  relaxation of the L2 projection of Hibler's law with e = 2 (the listings'
  constants) evaluated from an anisotropic, non-constant strain rate;
* one subcycle is strain -> stress -> divergence -> velocity with the NEW
  stress (Eq. (si:mevp): sigma^p from v^(p-1), then v^p from sigma^p);
* from rest, the first subcycle moves ice down the pressure gradient with the
  closed-form speed of a piecewise-constant pressure field.
"""
import numpy as np
import pytest

from synth_inputs import make_domain, random_state, uniform_vertices


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def interior_mask(nx, ny):
    NX, NY = 2 * nx + 1, 2 * ny + 1
    j = np.arange(NX * NY)
    ix, iy = j % NX, j // NX
    return (ix > 0) & (iy > 0) & (ix < NX - 1) & (iy < NY - 1)


# --------------------------------------------------------------------------- velocity
@pytest.mark.parametrize("f_cor", [0.0, 1.46e-4])
def test_velocity_update_solves_the_lumped_momentum_balance(oracle_mod, f_cor):
    """v^p returned by the velocity update satisfies, at every interior node,
      (M^H/dt) [beta (v^p - v^{p-1}) + v^p - v^n]
          = F + m^A tau_a + m^A rho_o C_o |v_o - v^{p-1}| (v_o - v^p) - f M^H k x v^p,
    checked as a residual (not by re-deriving the 2x2 solve), with a random
    nodal force of the size of the other terms, so that its sign and its
    component routing matter; v = 0 on the boundary."""
    O = oracle_mod
    p = O.Params(f_cor=f_cor, beta=50.0)
    d = make_domain(5, 4, 6, 1, seed=41, h=3000.0, perturb=0.15)
    m = O.Mesh(d.nx, d.ny, 6, 1, d.vertices)
    rng = np.random.default_rng(42)
    MH, mA = m.node_masses(p, d.H, d.A)
    tau = m.air_stress(p, d.wind)
    vprev = rng.normal(0, 0.05, (2, m.nn))
    vn = rng.normal(0, 0.05, (2, m.nn))
    ocean = rng.normal(0, 0.1, (2, m.nn))
    scale = np.abs(MH / p.dt * vn).max()
    F = rng.normal(0, 1.0, (2, m.nn)) * scale
    v = m.velocity(p, F, MH, mA, tau, ocean, vn, vprev)
    inner = interior_mask(d.nx, d.ny)
    drag = p.rho_o * p.C_o * np.hypot(ocean[0] - vprev[0], ocean[1] - vprev[1])
    kxv = np.stack([-v[1], v[0]])
    res = (MH / p.dt * (p.beta * (v - vprev) + v - vn) - F - mA * tau
           - mA * drag * (ocean - v) + f_cor * MH * kxv)
    terms = np.abs(F) + np.abs(MH / p.dt * (p.beta + 1) * v) + np.abs(mA * tau)
    assert (np.abs(res[:, inner]) <= 1e-13 * terms[:, inner].max()).all()
    assert (v[:, ~inner] == 0).all()
    # the force is not negligible in the balance: it moves v by O(1) of itself
    v0 = m.velocity(p, np.zeros_like(F), MH, mA, tau, ocean, vn, vprev)
    assert rel(v[:, inner], v0[:, inner]) > 0.1


def test_nodal_force_accelerates_along_itself(oracle_mod):
    """Ice at rest with no drag and no Coriolis: v^p = F dt / (M^H (1 + beta)),
    i.e. parallel to F with a positive factor (a force pushes the ice its way)."""
    O = oracle_mod
    p = O.Params(C_a=0.0, C_o=0.0, f_cor=0.0)
    m = O.Mesh(4, 3, 6, 1, uniform_vertices(4, 3, 2000.0))
    MH, mA = m.node_masses(p, np.full((1, m.ne), 1.5), np.full((1, m.ne), 0.9))
    rng = np.random.default_rng(5)
    F = rng.normal(0, 1e3, (2, m.nn))
    z = np.zeros((2, m.nn))
    v = m.velocity(p, F, MH, mA, z, z, z, z)
    inner = interior_mask(4, 3)
    np.testing.assert_allclose(v[:, inner], (F * p.dt / (MH * (1 + p.beta)))[:, inner], rtol=1e-14)


# --------------------------------------------------------------------------- stress
def hibler_e2(e11, e12, e22, P, dmin):
    """Hibler's viscous-plastic law with ellipse ratio e = 2 (the constants of
    the stress listings): zeta = P/(2 Delta), eta = zeta/e^2,
    sigma = 2 eta eps + (zeta - eta) tr(eps) I - P/2 I."""
    ecc2 = 4.0
    D = np.sqrt(dmin ** 2 + (e11 ** 2 + e22 ** 2) * (1 + 1 / ecc2) + 4 / ecc2 * e12 ** 2
                + 2 * e11 * e22 * (1 - 1 / ecc2))
    zeta = P / (2 * D)
    eta = zeta / ecc2
    tr = e11 + e22
    return (2 * eta * e11 + (zeta - eta) * tr - P / 2, 2 * eta * e12,
            2 * eta * e22 + (zeta - eta) * tr - P / 2)


@pytest.mark.parametrize("ns,na,relax_form", [(3, 1, 0), (6, 3, 0), (8, 6, 0), (6, 3, 1)])
def test_stress_update_every_component_and_coefficient(oracle_mod, ns, na, relax_form):
    """S <- fac S_0 + ainv Pi_e(sigma(e)) per component and per DG coefficient,
    from a strain rate whose three components differ in size and vary inside
    the cell, with a random S_0 of the same size as the new stress and the
    ice clamps active; Pi_e and the Gauss values come from the separately
    pinned projection and evaluation."""
    O = oracle_mod
    p = O.Params(alpha=7.0, relax_form=relax_form)
    d = make_domain(4, 3, ns, na, seed=43, h=1500.0, perturb=0.15, ho_amp=0.4)
    m = O.Mesh(d.nx, d.ny, ns, na, d.vertices)
    rng = np.random.default_rng(44)
    decay = np.array([1.0, 0.6, 0.6, 0.3, 0.3, 0.3, 0.2, 0.2])[:ns]
    E = rng.normal(0, 1, (3, ns, m.ne)) * decay[None, :, None]
    E[0] *= 3e-7
    E[1] *= 1e-7
    E[2] *= -5e-8
    S0 = rng.normal(0, 2e4, (3, ns, m.ne))
    H, A = d.H.copy(), d.A.copy()
    A[0, ::3] = 1.1                                  # concentration above one in some cells
    H[0, 1] = -0.2                                   # and a negative thickness in one
    S = m.stress(p, E, H, A, S0)
    psiA = O.tables(ns, na)[3]                       # [na][nG]
    h = np.maximum(0.0, np.einsum("kq,ke->qe", psiA, H))
    a = np.minimum(1.0, np.maximum(0.0, np.einsum("kq,ke->qe", psiA, A)))
    assert (h == 0).any() and (a == 1).any()        # both clamps bite somewhere
    P = p.Pstar * h * np.exp(-p.C * (1 - a))
    e11, e12, e22 = m.eval_gauss(E)
    s = np.stack(hibler_e2(e11, e12, e22, P, p.DeltaMin))
    if relax_form == 0:
        fac, ainv = 1 - 1 / p.alpha, 1 / p.alpha
    else:
        fac, ainv = p.alpha / (1 + p.alpha), 1 / (1 + p.alpha)
    expect = fac * S0 + ainv * m.project(s)
    for c in range(3):
        for k in range(ns):
            assert rel(S[c, k], expect[c, k]) < 1e-11, (c, k)
    # the strain components are not interchangeable on this input
    swapped = fac * S0 + ainv * m.project(np.stack(hibler_e2(e22, e12, e11, P, p.DeltaMin)))
    assert rel(swapped[0], expect[0]) > 1e-3


# --------------------------------------------------------------------------- composition
@pytest.mark.parametrize("ns", [3, 6])
def test_subcycle_is_strain_stress_divergence_velocity_with_new_stress(oracle_mod, ns):
    """One subcycle equals velocity(divergence(stress(strain(v^{p-1}), S^{p-1})))
    with the per-step masses and air stress, i.e. the divergence reads the
    stress just updated (Eq. (si:mevp)); two subcycles chain it; a time step
    snapshots v^n = v at its start."""
    O = oracle_mod
    p = O.Params()
    d = make_domain(6, 5, ns, 1, seed=45, h=4000.0, perturb=0.1)
    m = O.Mesh(d.nx, d.ny, ns, 1, d.vertices)
    v0, S0 = random_state(d.nx, d.ny, ns, seed=46)
    vn = random_state(d.nx, d.ny, ns, seed=47)[0]
    MH, mA = m.node_masses(p, d.H, d.A)
    tau = m.air_stress(p, d.wind)

    def by_hand(v, S):
        S = m.stress(p, m.strain(v), d.H, d.A, S)
        v = m.velocity(p, m.divergence(S), MH, mA, tau, d.ocean, vn, v)
        return v, S

    v1, S1 = by_hand(v0, S0)
    v2, S2 = by_hand(v1, S1)
    a1 = m.subcycles(p, d.H, d.A, d.wind, d.ocean, vn, v0, S0, 1)
    a2 = m.subcycles(p, d.H, d.A, d.wind, d.ocean, vn, v0, S0, 2)
    assert np.array_equal(a1[0], v1) and np.array_equal(a1[1], S1)
    assert np.array_equal(a2[0], v2) and np.array_equal(a2[1], S2)
    # with the old stress the velocity would differ at first order here
    v_old = m.velocity(p, m.divergence(S0), MH, mA, tau, d.ocean, vn, v0)
    assert rel(v_old, v1) > 1e-3
    # a time step: v^n is the velocity at its start
    st = m.step(p, d.H, d.A, d.wind, d.ocean, v0, S0, 2)
    sc = m.subcycles(p, d.H, d.A, d.wind, d.ocean, v0, v0, S0, 2)
    assert np.array_equal(st[0], sc[0]) and np.array_equal(st[1], sc[1])


def test_first_subcycle_from_rest_follows_the_pressure_gradient(oracle_mod):
    """Ice at rest (v = 0, S = 0), no wind, no ocean, no Coriolis, A = 1 and H
    constant per cell column. The first subcycle sees zero strain, so the new
    stress is sigma = -P_e/(2 alpha) I per cell (exactly: the projection keeps
    constants). Its weak divergence at a CG2 node on the vertical edge between
    columns i-1 and i is F_x = h_y W (P_{i-1} - P_i) / (2 alpha), with
    W = 2/3 at an edge midpoint and 1/3 at a vertex (the integrals of the 1D
    quadratic Lagrange functions along the edge, from the cells above and
    below), zero at column-interior nodes, and F_y = 0. With the lumped mass
    M^H = rho_i sum_e H_e |K| w_c w_b (1D weights 1/6, 2/3, 1/6) the new
    velocity is v_x = F_x dt / (M^H (1 + beta)): ice moves from thick to thin."""
    O = oracle_mod
    p = O.Params(f_cor=0.0)
    nx, ny, hx, hy = 6, 4, 3000.0, 2000.0
    m = O.Mesh(nx, ny, 6, 1, uniform_vertices(nx, ny, hx, hy))
    Hcol = np.array([0.6, 0.9, 1.7, 1.7, 1.2, 2.0])
    H = np.tile(Hcol, ny)[None, :]
    A = np.ones((1, m.ne))
    z = np.zeros((2, m.nn))
    v, S = m.step(p, H, A, z, z, z, np.zeros((3, 6, m.ne)), 1)
    Pcol = p.Pstar * Hcol
    NX = 2 * nx + 1
    w1 = np.array([1 / 6, 2 / 3, 1 / 6])
    vx_expect = np.zeros((2 * ny + 1, NX))
    for iy in range(1, 2 * ny):
        for ix in range(1, NX - 1):
            # lumped mass: every cell touching the node contributes rho_i H |K| w_c w_b
            MH = 0.0
            for ey in range(ny):
                for ex in range(nx):
                    c, b = ix - 2 * ex, iy - 2 * ey
                    if 0 <= c <= 2 and 0 <= b <= 2:
                        MH += p.rho_i * Hcol[ex] * hx * hy * w1[c] * w1[b]
            if ix % 2 == 0:
                i = ix // 2
                W = 2 / 3 if iy % 2 else 1 / 3
                Fx = hy * W * (Pcol[i - 1] - Pcol[i]) / (2 * p.alpha)
                vx_expect[iy, ix] = Fx * p.dt / (MH * (1 + p.beta))
    vx = v[0].reshape(2 * ny + 1, NX)
    vy = v[1].reshape(2 * ny + 1, NX)
    scale = np.abs(vx_expect).max()
    assert scale > 1e-6  # m/s: the pressure jumps move the ice (1/alpha of the full stress)
    assert np.abs(vx - vx_expect).max() < 1e-12 * scale
    assert np.abs(vy).max() < 1e-12 * scale
    np.testing.assert_allclose(S[0, 0], -p.Pstar * H[0] / (2 * p.alpha), rtol=1e-13)


def test_ice_free_interior_nodes_are_held_at_rest(oracle_mod):
    """At an interior node with no ice (M^H = m^A = 0) the lumped balance has
    no mass on either side and no drag: the velocity update holds the node at
    rest in both components, whatever v^(p-1), v^n and the nodal force (the
    library's reading of the degenerate node); every other interior node still
    satisfies the balance."""
    O = oracle_mod
    p = O.Params(f_cor=1.46e-4, beta=50.0)
    d = make_domain(5, 4, 6, 1, seed=43, h=3000.0, perturb=0.1)
    m = O.Mesh(d.nx, d.ny, 6, 1, d.vertices)
    rng = np.random.default_rng(44)
    MH, mA = m.node_masses(p, d.H, d.A)
    inner = interior_mask(d.nx, d.ny)
    free = np.flatnonzero(inner)[[0, 7, 20, 33]]
    MH[free] = 0.0
    mA[free] = 0.0
    tau = m.air_stress(p, d.wind)
    vprev = rng.normal(0, 0.05, (2, m.nn))
    vn = rng.normal(0, 0.05, (2, m.nn))
    ocean = rng.normal(0, 0.1, (2, m.nn))
    F = rng.normal(0, 1.0, (2, m.nn)) * np.abs(MH / p.dt * vn).max()
    v = m.velocity(p, F, MH, mA, tau, ocean, vn, vprev)
    assert (v[:, free] == 0).all()
    assert (v[:, ~inner] == 0).all()
    rest = inner.copy()
    rest[free] = False
    drag = p.rho_o * p.C_o * np.hypot(ocean[0] - vprev[0], ocean[1] - vprev[1])
    kxv = np.stack([-v[1], v[0]])
    res = (MH / p.dt * (p.beta * (v - vprev) + v - vn) - F - mA * tau
           - mA * drag * (ocean - v) + p.f_cor * MH * kxv)
    terms = np.abs(F) + np.abs(MH / p.dt * (p.beta + 1) * v) + np.abs(mA * tau)
    assert (np.abs(res[:, rest]) <= 1e-13 * terms[:, rest].max()).all()


def test_zero_subcycles_leave_the_state_unchanged(oracle_mod):
    """n_sub = 0 is a valid call that changes nothing; n_sub < 0 is rejected."""
    O = oracle_mod
    p = O.Params()
    d = make_domain(4, 3, 6, 1, seed=45, h=2000.0)
    m = O.Mesh(d.nx, d.ny, 6, 1, d.vertices)
    v0, S0 = random_state(d.nx, d.ny, 6, seed=46)
    v, S = m.subcycles(p, d.H, d.A, d.wind, d.ocean, v0, v0, S0, 0)
    assert np.array_equal(v, v0) and np.array_equal(S, S0)
    v, S = m.step(p, d.H, d.A, d.wind, d.ocean, v0, S0, 0)
    assert np.array_equal(v, v0) and np.array_equal(S, S0)
    with pytest.raises(RuntimeError):
        m.subcycles(p, d.H, d.A, d.wind, d.ocean, v0, v0, S0, -1)
