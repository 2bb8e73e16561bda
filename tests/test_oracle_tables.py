"""Pins of the oracle's reference-element tables against textbook values.

Gauss rule: NGP x NGP tensor Gauss-Legendre with NGP from the number of stress
dofs (appendix listing of the paper). DG basis: the orthogonal scaled-Legendre
reading; CG2: biquadratic Lagrange (Sec. 2.1 names higher-order CG velocity and
tensor-valued DG stress).
"""
import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("ns,ngp", [(3, 2), (6, 3), (8, 3)])
def test_gauss_rule_matches_tabulated(oracle_mod, ns, ngp):
    g = json.load(open(os.path.join(GOLD, "gauss_legendre.json")))[f"n{ngp}"]
    gp, gw, *_ = oracle_mod.tables(ns)
    # map [-1,1] -> [0,1]
    np.testing.assert_allclose(gp, (1.0 + np.array(g["x"])) / 2.0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(gw, np.array(g["w"]) / 2.0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("ns,ngp", [(3, 2), (6, 3)])
def test_gauss_exactness_degree(oracle_mod, ns, ngp):
    gp, gw, *_ = oracle_mod.tables(ns)
    for k in range(2 * ngp):
        assert abs(np.dot(gw, gp ** k) - 1.0 / (k + 1)) < 1e-15
    # first degree that is not integrated exactly
    assert abs(np.dot(gw, gp ** (2 * ngp)) - 1.0 / (2 * ngp + 1)) > 1e-6


@pytest.mark.parametrize("ns", [3, 6, 8])
def test_dg_basis_orthogonal_with_known_norms(oracle_mod, ns):
    gp, gw, psiS, *_ = oracle_mod.tables(ns)
    ngp = len(gp)
    W = np.outer(gw, gw).ravel()  # q = qy*ngp + qx
    M = (psiS * W) @ psiS.T
    norms = np.array([1, 1 / 12, 1 / 12, 1 / 180, 1 / 144, 1 / 180, 1 / 2160, 1 / 2160])[:ns]
    np.testing.assert_allclose(M, np.diag(norms), atol=1e-15)
    # values at the Gauss points: psi_1 = xi - 1/2, psi_2 = eta - 1/2
    xi = np.tile(gp, ngp)
    eta = np.repeat(gp, ngp)
    np.testing.assert_allclose(psiS[0], 1.0)
    np.testing.assert_allclose(psiS[1], xi - 0.5, atol=1e-16)
    np.testing.assert_allclose(psiS[2], eta - 0.5, atol=1e-16)


def test_q2_lagrange_integrals_and_partition_of_unity(oracle_mod):
    gp, gw, psiS, psiA, phi, dxi, deta = oracle_mod.tables(6)
    W = np.outer(gw, gw).ravel()
    one_d = np.array([1 / 6, 2 / 3, 1 / 6])
    expect = np.array([one_d[a % 3] * one_d[a // 3] for a in range(9)])  # 1/36, 1/9, 4/9
    np.testing.assert_allclose(phi @ W, expect, atol=1e-16)
    np.testing.assert_allclose(phi.sum(0), 1.0, atol=1e-15)
    np.testing.assert_allclose(dxi.sum(0), 0.0, atol=1e-14)
    np.testing.assert_allclose(deta.sum(0), 0.0, atol=1e-14)
    # Lagrange property at the nodes: compare with the values at the 3x3 Gauss points of
    # an independent evaluation of (1-t)(1-2t), 4t(1-t), t(2t-1)
    L = lambda t: np.array([(1 - t) * (1 - 2 * t), 4 * t * (1 - t), t * (2 * t - 1)])
    xi, eta = np.tile(gp, 3), np.repeat(gp, 3)
    ref = np.array([L(xi)[a % 3] * L(eta)[a // 3] for a in range(9)])
    np.testing.assert_allclose(phi, ref, atol=1e-15)


def test_listing_constants_golden(oracle_mod):
    """The oracle's pointwise stress reproduces the constants printed in the listings."""
    gold = json.load(open(os.path.join(GOLD, "stress_listing_constants.json")))
    O = oracle_mod
    from synth_inputs import uniform_vertices
    m = O.Mesh(1, 1, 6, 1, uniform_vertices(1, 1, 1000.0))
    p = O.Params()
    rng = np.random.default_rng(5)
    E = rng.normal(0, 1e-6, (3, 6, 1))
    H = np.array([[1.3]])
    A = np.array([[0.93]])
    s, P, D = m.stress_gauss(p, E, H, A)
    e = m.eval_gauss(E)[:, :, 0]
    Pg = p.Pstar * 1.3 * np.exp(-gold["C"] * (1 - 0.93))
    d = gold["delta_sq"]
    Dg = np.sqrt(p.DeltaMin ** 2 + d["e11e11_plus_e22e22"] * (e[0] ** 2 + e[2] ** 2)
                 + d["e11e22"] * e[0] * e[2] + d["e12e12"] * e[1] ** 2)
    PD = Pg / Dg
    np.testing.assert_allclose(P[:, 0], Pg, rtol=1e-14)
    np.testing.assert_allclose(D[:, 0], Dg, rtol=1e-14)
    np.testing.assert_allclose(s[0, :, 0], PD * (gold["s11"]["e11"] * e[0] + gold["s11"]["e22"] * e[2]) + gold["s11"]["P"] * Pg, rtol=1e-13)
    np.testing.assert_allclose(s[1, :, 0], PD * gold["s12"]["e12"] * e[1], rtol=1e-13)
    np.testing.assert_allclose(s[2, :, 0], PD * (gold["s22"]["e22"] * e[2] + gold["s22"]["e11"] * e[0]) + gold["s22"]["P"] * Pg, rtol=1e-13)


@pytest.mark.parametrize("ns", [3, 6])
def test_q2_gradients_differentiate_the_q2_space_exactly(oracle_mod, ns):
    """The reference gradient tables differentiate every function of the Q2
    space exactly: for f = xi^i eta^j (i, j <= 2), sum_a f(node_a) dphi_a/dxi
    at each Gauss point is df/dxi there, likewise for eta (node a = 3 b + c at
    (c/2, b/2))."""
    gp, gw, psiS, psiA, phi, dxi, deta = oracle_mod.tables(ns)
    ngp = len(gp)
    xq, eq = np.tile(gp, ngp), np.repeat(gp, ngp)
    xa = np.array([(a % 3) / 2 for a in range(9)])
    ea = np.array([(a // 3) / 2 for a in range(9)])
    for i in range(3):
        for j in range(3):
            f = xa ** i * ea ** j
            dfx = i * xq ** max(i - 1, 0) * eq ** j
            dfe = j * xq ** i * eq ** max(j - 1, 0)
            np.testing.assert_allclose(f @ dxi, dfx, atol=1e-14)
            np.testing.assert_allclose(f @ deta, dfe, atol=1e-14)
