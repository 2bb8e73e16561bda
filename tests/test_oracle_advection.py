"""Pins of the oracle's DG upwind advection of H and A (Sec. 2, Eq. (si:ad);
reading R14 in oracle/mevp_oracle.c): rest, conservation, constant
preservation under a divergence-free field, exact translation of polynomial
profiles, and an exact-arithmetic rate on a 2x2 mesh."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from brute_fe import AffineMesh, advect_rate
from synth_inputs import make_domain, perturbed_vertices, uniform_vertices


def _cell_integrals(m, H):
    """sum_e int_K H over the mesh with a 3x3 Gauss rule of independent code."""
    x = np.array([0.5 - 0.5 * np.sqrt(0.6), 0.5, 0.5 + 0.5 * np.sqrt(0.6)])
    w = np.array([5 / 18, 4 / 9, 5 / 18])
    V = m.vertices
    X = V[0].reshape(m.ny + 1, m.nx + 1)
    Y = V[1].reshape(m.ny + 1, m.nx + 1)
    tot = 0.0
    for ey in range(m.ny):
        for ex in range(m.nx):
            x0, x1, x2, x3 = X[ey, ex], X[ey, ex + 1], X[ey + 1, ex], X[ey + 1, ex + 1]
            y0, y1, y2, y3 = Y[ey, ex], Y[ey, ex + 1], Y[ey + 1, ex], Y[ey + 1, ex + 1]
            e = ey * m.nx + ex
            for qy in range(3):
                for qx in range(3):
                    xi, eta = x[qx], x[qy]
                    J00 = (1 - eta) * (x1 - x0) + eta * (x3 - x2)
                    J01 = (1 - xi) * (x2 - x0) + xi * (x3 - x1)
                    J10 = (1 - eta) * (y1 - y0) + eta * (y3 - y2)
                    J11 = (1 - xi) * (y2 - y0) + xi * (y3 - y1)
                    s, t = xi - 0.5, eta - 0.5
                    basis = [1, s, t, s * s - 1 / 12, s * t, t * t - 1 / 12][:m.na]
                    hv = sum(H[k, e] * basis[k] for k in range(m.na))
                    tot += w[qx] * w[qy] * (J00 * J11 - J01 * J10) * hv
    return tot


def _interior_mask(nx, ny):
    NX, NY = 2 * nx + 1, 2 * ny + 1
    ix, iy = np.arange(NX * NY) % NX, np.arange(NX * NY) // NX
    return (ix > 0) & (iy > 0) & (ix < NX - 1) & (iy < NY - 1)


@pytest.mark.parametrize("na", [1, 3, 6])
def test_rest_leaves_fields_unchanged(oracle_mod, na):
    d = make_domain(7, 6, 6, na, seed=3, h=2e3, perturb=0.1, ho_amp=0.2)
    m = oracle_mod.Mesh(7, 6, 6, na, d.vertices)
    H, A = m.advect(120.0, np.zeros((2, m.nn)), d.H, d.A)
    # the Runge-Kutta stage blends (3/4 U + 1/4 U, 1/3 U + 2/3 U) round, nothing else
    assert np.abs(H - d.H).max() <= 4e-16 * np.abs(d.H).max()
    assert np.abs(A - d.A).max() <= 4e-16 * np.abs(d.A).max()


@pytest.mark.parametrize("na", [1, 3, 6])
def test_mass_is_conserved(oracle_mod, na):
    """v = 0 on the boundary: no flux leaves the domain, and the upwind fluxes
    cancel pairwise across interior edges."""
    d = make_domain(9, 7, 6, na, seed=4, h=2e3, perturb=0.15, ho_amp=0.2)
    m = oracle_mod.Mesh(9, 7, 6, na, d.vertices)
    rng = np.random.default_rng(1)
    v = rng.normal(0, 0.3, (2, m.nn)) * _interior_mask(9, 7)
    H, A = d.H, d.A
    m0 = _cell_integrals(m, H)
    for _ in range(3):
        H, A = m.advect(600.0, v, H, A)
    assert np.abs(H - d.H).max() > 1e-4  # something moved
    assert abs(_cell_integrals(m, H) - m0) < 1e-12 * abs(m0)


@pytest.mark.parametrize("na", [1, 3, 6])
def test_constant_preserved_by_rotation(oracle_mod, na):
    """A constant field under the divergence-free rotation v = w (-(y-yc), x-xc)
    stays constant (the rate of a constant is -U int div v psi = 0)."""
    nx, ny, h = 6, 5, 1000.0
    m = oracle_mod.Mesh(nx, ny, 6, na, uniform_vertices(nx, ny, h))
    NX = 2 * nx + 1
    ix, iy = np.arange(m.nn) % NX, np.arange(m.nn) // NX
    x, y = ix * h / 2, iy * h / 2
    om = 2e-5
    v = np.stack([-om * (y - 2500.0), om * (x - 3000.0)])
    H = np.zeros((na, m.ne))
    H[0] = 1.7
    L = m.advect_rate(v, H)
    assert np.abs(L).max() < 1e-15
    H2, _ = m.advect(300.0, v, H, H)
    assert np.abs(H2 - H).max() < 1e-14


@pytest.mark.parametrize("na,deg", [(3, 1), (6, 2)])
def test_translation_of_polynomial_profile_is_exact(oracle_mod, na, deg):
    """Uniform velocity c: a profile H = a + b x (+ d x^2) in the DG space moves
    exactly (upwind sees no jump, three-stage RK3 integrates a polynomial of
    degree <= 3 in time exactly)."""
    nx, ny, h = 12, 3, 1000.0
    m = oracle_mod.Mesh(nx, ny, 6, na, uniform_vertices(nx, ny, h))
    c, dt = 1.5, 120.0
    a, b, dd = 0.8, 2e-4, (3e-8 if deg == 2 else 0.0)
    ex = np.tile(np.arange(nx), ny)

    def coefs(shift):
        xc = (ex + 0.5) * h - shift
        H = np.zeros((na, m.ne))
        # H(x) = a + b x + d x^2 around the cell centre, x - xc = h (xi - 1/2):
        # a + b xc + d xc^2 + (b + 2 d xc) h s + d h^2 s^2, s^2 = (s^2 - 1/12) + 1/12
        H[0] = a + b * xc + dd * xc ** 2 + dd * h * h / 12.0
        H[1] = (b + 2 * dd * xc) * h
        if na == 6:
            H[3] = dd * h * h
        return H

    v = np.stack([np.full(m.nn, c), np.zeros(m.nn)])
    H1, _ = m.advect(dt, v, coefs(0.0), coefs(0.0))
    exact = coefs(c * dt)
    # the inflow boundary takes the cell's own trace, which for a profile in the
    # DG space is the exact solution's trace: every cell is exact
    assert np.abs(H1 - exact).max() < 1e-13 * np.abs(exact).max()
    assert np.abs(H1 - coefs(0.0)).max() > 1e-3 * np.abs(exact).max()  # it moved


@pytest.mark.parametrize("na", [1, 3, 6])
def test_rate_matches_exact_assembly(oracle_mod, na):
    """Exact rational rate on a 2x2 sheared mesh (tests/brute_fe.py): v keeps one
    sign of v.n on every edge so the upwind side is fixed, and (for n_a = 6) is
    linear so that the 3-point edge rule is exact."""
    HX, HY, SH = 3, 2, 1
    bm = AffineMesh(2, 2, HX, HY, SH)
    xs, ys = bm.vertices()
    V = np.array([[float(x) for x in xs], [float(y) for y in ys]])
    m = oracle_mod.Mesh(2, 2, 6, na, V)
    rng = np.random.default_rng(na)
    NX = 5
    vx, vy = [], []
    for j in range(bm.nn):
        ix, iy = j % NX, j // NX
        x = Fr(ix * HX + iy * SH, 2)
        y = Fr(iy * HY, 2)
        if na == 6:
            vx.append(Fr(3, 2) + x / 20 - y / 30)
            vy.append(Fr(1, 2) - x / 40 + y / 25)
        else:
            vx.append(Fr(3, 2) + Fr(int(rng.integers(-2, 3)), 16))
            vy.append(Fr(1, 2) + Fr(int(rng.integers(-2, 3)), 16))
    U = [[Fr(int(z), 8) for z in rng.integers(-9, 10, bm.ne)] for _ in range(na)]
    exact = advect_rate(bm, vx, vy, U, na)
    L = m.advect_rate(np.array([[float(z) for z in vx], [float(z) for z in vy]]),
                      np.array([[float(z) for z in r] for r in U]))
    ref = np.array([[float(z) for z in r] for r in exact])
    assert np.abs(L - ref).max() < 1e-13 * np.abs(ref).max()


def _sheared_vertices(nx, ny, h, sx, sy):
    """Parallelogram cells with edge vectors (h, sy h) and (sx h, h): both
    off-diagonal Jacobian entries are non-zero."""
    iy, ix = np.meshgrid(np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    return np.stack([(ix + sx * iy).ravel() * h, (iy + sy * ix).ravel() * h]).astype(np.float64)


@pytest.mark.parametrize("na", [3, 6])
@pytest.mark.parametrize("cells", ["sheared", "bilinear"])
def test_free_stream_rate_is_zero_on_general_cells(oracle_mod, na, cells):
    """A constant field carried by a constant velocity has a zero rate in every
    cell: the volume term integrates U v.grad(psi_k) exactly (a polynomial of
    low degree after the Jacobian's adjugate) and equals the sum of the edge
    fluxes, each edge's upwind value being the same constant (own trace on the
    domain boundary). The cells have both off-diagonal Jacobian entries
    non-zero, so every term of grad psi = J^-T (dpsi/dxi, dpsi/deta) enters."""
    nx, ny, h = 6, 5, 1000.0
    if cells == "sheared":
        V = _sheared_vertices(nx, ny, h, 0.3, 0.2)
    else:
        V = perturbed_vertices(nx, ny, h, amp=0.2, seed=5)
    m = oracle_mod.Mesh(nx, ny, 6, na, V)
    U = np.zeros((na, m.ne))
    U[0] = 0.9
    ux, uy = 0.4, -0.25
    v = np.stack([np.full(m.nn, ux), np.full(m.nn, uy)])
    L = m.advect_rate(v, U)
    scale = 0.9 * np.hypot(ux, uy) / h
    assert np.abs(L).max() <= 1e-12 * scale
    # a non-constant field does move (the test is not vacuous)
    U2 = U.copy()
    U2[1] = 0.2
    assert np.abs(m.advect_rate(v, U2)).max() > 1e-3 * scale


@pytest.mark.parametrize("na", [1, 3])
def test_both_fields_advected_alike(oracle_mod, na):
    """H and A go through the same scheme, each on its own: swapping them at
    the input swaps the outputs bit for bit, both move under a non-zero
    velocity, and both keep their cell integrals."""
    d = make_domain(7, 6, 6, na, seed=7, h=2e3, perturb=0.1, ho_amp=0.2)
    m = oracle_mod.Mesh(7, 6, 6, na, d.vertices)
    rng = np.random.default_rng(8)
    v = rng.normal(0, 0.3, (2, m.nn)) * _interior_mask(7, 6)
    H1, A1 = m.advect(600.0, v, d.H, d.A)
    A2, H2 = m.advect(600.0, v, d.A, d.H)
    assert np.array_equal(H1, H2) and np.array_equal(A1, A2)
    for U0, U1 in ((d.H, H1), (d.A, A1)):
        assert np.abs(U1 - U0).max() > 1e-6 * np.abs(U0).max()
        m0 = _cell_integrals(m, U0)
        assert abs(_cell_integrals(m, U1) - m0) < 1e-12 * abs(m0)
