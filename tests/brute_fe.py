"""Exact-arithmetic finite elements on small parallelogram meshes (test helper).

Independent of the oracle: polynomials in the reference coordinates (xi, eta)
with Fraction coefficients, integrated exactly over [0,1]^2 (no quadrature).
Used to assemble, densely and globally, the CG2 lumped masses, the projected
strain operator and the divergence operator on a 2x2 mesh, which the oracle's
Gauss-quadrature element loops must reproduce to rounding.
"""
from __future__ import annotations

from fractions import Fraction as Fr
from itertools import product


class Poly:
    """Polynomial in (xi, eta): {(i, j): coefficient of xi^i eta^j}."""

    def __init__(self, terms=None):
        self.t = {k: Fr(v) for k, v in (terms or {}).items() if v != 0}

    @staticmethod
    def const(c):
        return Poly({(0, 0): c})

    def __add__(self, o):
        o = o if isinstance(o, Poly) else Poly.const(o)
        r = dict(self.t)
        for k, v in o.t.items():
            r[k] = r.get(k, Fr(0)) + v
        return Poly(r)

    __radd__ = __add__

    def __neg__(self):
        return Poly({k: -v for k, v in self.t.items()})

    def __sub__(self, o):
        return self + (-(o if isinstance(o, Poly) else Poly.const(o)))

    def __mul__(self, o):
        if not isinstance(o, Poly):
            return Poly({k: v * Fr(o) for k, v in self.t.items()})
        r = {}
        for (a, b), u in self.t.items():
            for (c, d), w in o.t.items():
                r[(a + c, b + d)] = r.get((a + c, b + d), Fr(0)) + u * w
        return Poly(r)

    __rmul__ = __mul__

    def dxi(self):
        return Poly({(i - 1, j): v * i for (i, j), v in self.t.items() if i > 0})

    def deta(self):
        return Poly({(i, j - 1): v * j for (i, j), v in self.t.items() if j > 0})

    def integral(self):
        """Exact integral over the unit square."""
        return sum((v / ((i + 1) * (j + 1)) for (i, j), v in self.t.items()), Fr(0))


XI = Poly({(1, 0): 1})
ETA = Poly({(0, 1): 1})


def lagrange_1d(var):
    one = Poly.const(1)
    return [(one - var) * (one - 2 * var), 4 * var * (one - var), var * (2 * var - one)]


def q2_basis():
    Lx, Ly = lagrange_1d(XI), lagrange_1d(ETA)
    return [Lx[a % 3] * Ly[a // 3] for a in range(9)]


def dg_basis(n):
    s = XI - Fr(1, 2)
    t = ETA - Fr(1, 2)
    b = [Poly.const(1), s, t, s * s - Fr(1, 12), s * t, t * t - Fr(1, 12),
         (s * s - Fr(1, 12)) * t, s * (t * t - Fr(1, 12))]
    return b[:n]


class AffineMesh:
    """nx x ny parallelograms: vertex (ix, iy) at (ix*hx + iy*shear, iy*hy)."""

    def __init__(self, nx, ny, hx, hy, shear):
        self.nx, self.ny = nx, ny
        self.hx, self.hy, self.sh = Fr(hx), Fr(hy), Fr(shear)
        self.det = self.hx * self.hy
        self.phi = q2_basis()

    @property
    def ne(self):
        return self.nx * self.ny

    @property
    def nn(self):
        return (2 * self.nx + 1) * (2 * self.ny + 1)

    def node(self, e, a):
        ex, ey = e % self.nx, e // self.nx
        return (2 * ey + a // 3) * (2 * self.nx + 1) + 2 * ex + a % 3

    # x = x0 + hx xi + sh eta, y = y0 + hy eta  =>  d/dx = d/dxi / hx,
    # d/dy = (-sh d/dxi + hx d/deta) / (hx hy)
    def ddx(self, p):
        return p.dxi() * (1 / self.hx)

    def ddy(self, p):
        return (p.dxi() * (-self.sh) + p.deta() * self.hx) * (1 / self.det)

    def lumped(self, coef, rho=1):
        """sum_e int rho * (sum_k coef[k][e] psi_k) phi_j dx for each node j (no clamp)."""
        na = len(coef)
        psi = dg_basis(na)
        out = [Fr(0)] * self.nn
        for e in range(self.ne):
            f = sum((psi[k] * coef[k][e] for k in range(na)), Poly())
            for a in range(9):
                out[self.node(e, a)] += (f * self.phi[a]).integral() * self.det * rho
        return out

    def strain(self, vx, vy, ns):
        """Projected strain coefficients E[c][k][e] (c: 11, 12, 22), exact."""
        psi = dg_basis(ns)
        norms = [(p * p).integral() for p in psi]
        E = [[[Fr(0)] * self.ne for _ in range(ns)] for _ in range(3)]
        for e in range(self.ne):
            ux = sum((self.phi[a] * vx[self.node(e, a)] for a in range(9)), Poly())
            uy = sum((self.phi[a] * vy[self.node(e, a)] for a in range(9)), Poly())
            eps = [self.ddx(ux), (self.ddy(ux) + self.ddx(uy)) * Fr(1, 2), self.ddy(uy)]
            for c, k in product(range(3), range(ns)):
                E[c][k][e] = (psi[k] * eps[c]).integral() / norms[k]
        return E

    def divergence(self, S, ns):
        """F_j = -sum_e int sigma grad phi_j, exact; S[c][k][e]."""
        psi = dg_basis(ns)
        Fx = [Fr(0)] * self.nn
        Fy = [Fr(0)] * self.nn
        for e in range(self.ne):
            sg = [sum((psi[k] * S[c][k][e] for k in range(ns)), Poly()) for c in range(3)]
            for a in range(9):
                gx, gy = self.ddx(self.phi[a]), self.ddy(self.phi[a])
                j = self.node(e, a)
                Fx[j] -= (sg[0] * gx + sg[1] * gy).integral() * self.det
                Fy[j] -= (sg[1] * gx + sg[2] * gy).integral() * self.det
        return Fx, Fy

    def vertices(self):
        xs, ys = [], []
        for iy in range(self.ny + 1):
            for ix in range(self.nx + 1):
                xs.append(ix * self.hx + iy * self.sh)
                ys.append(iy * self.hy)
        return xs, ys


# ---------------------------------------------------------------------------
# DG upwind advection rate, exact (edges by exact 1D polynomial integrals)
# ---------------------------------------------------------------------------
def _pow_poly(base, n):
    """(base)^n for base a dict {power: coef} in one variable u."""
    out = {0: Fr(1)}
    for _ in range(n):
        nxt = {}
        for i, a in out.items():
            for j, b in base.items():
                nxt[i + j] = nxt.get(i + j, Fr(0)) + a * b
        out = nxt
    return out


def restrict(p, xi_of_u, eta_of_u):
    """p(xi(u), eta(u)) as {power: coef}; xi_of_u, eta_of_u are {power: coef}."""
    out = {}
    for (i, j), c in p.t.items():
        xi_p = _pow_poly(xi_of_u, i)
        eta_p = _pow_poly(eta_of_u, j)
        for a, ca in xi_p.items():
            for b, cb in eta_p.items():
                out[a + b] = out.get(a + b, Fr(0)) + c * ca * cb
    return out


def upoly_mul(*ps):
    out = {0: Fr(1)}
    for p in ps:
        nxt = {}
        for i, a in out.items():
            for j, b in p.items():
                nxt[i + j] = nxt.get(i + j, Fr(0)) + a * b
        out = nxt
    return out


def upoly_int(p):
    return sum((c / (i + 1) for i, c in p.items()), Fr(0))


def upoly_at(p, u):
    return sum((c * Fr(u) ** i for i, c in p.items()), Fr(0))


U_ = {1: Fr(1)}
ONE_ = {0: Fr(1)}
ZERO_ = {}
ONE_MINUS_U = {0: Fr(1), 1: Fr(-1)}
# edge ed traversed counter-clockwise: (xi(u), eta(u)) on this element and on the neighbour
EDGE_SELF = [(U_, ZERO_), (ONE_, U_), (ONE_MINUS_U, ONE_), (ZERO_, ONE_MINUS_U)]
EDGE_NB = [(U_, ONE_), (ZERO_, U_), (ONE_MINUS_U, ZERO_), (ONE_, ONE_MINUS_U)]
EDGE_NB_OFFSET = [(0, -1), (1, 0), (0, 1), (-1, 0)]
EDGE_VERTS = [(0, 1), (1, 3), (3, 2), (2, 0)]  # local vertices (0,0) (1,0) (0,1) (1,1)


def dg_grad(k_poly):
    return k_poly.dxi(), k_poly.deta()


def advect_rate(bm, vx, vy, U, na):
    """Exact L = M^-1 R of the DG upwind advection rate (reading R14 of the
    oracle), for v with one sign of v.n along every edge. U[k][e]."""
    psi = dg_basis(na)
    norms = [(p * p).integral() for p in psi]
    out = [[Fr(0)] * bm.ne for _ in range(na)]
    hx, hy, sh = bm.hx, bm.hy, bm.sh
    # vertex coordinates of the reference corners (relative): (0,0), (hx,0), (sh,hy), (hx+sh,hy)
    corner = [(Fr(0), Fr(0)), (hx, Fr(0)), (sh, hy), (hx + sh, hy)]
    for e in range(bm.ne):
        ex, ey = e % bm.nx, e // bm.nx
        ux = sum((bm.phi[a] * vx[bm.node(e, a)] for a in range(9)), Poly())
        uy = sum((bm.phi[a] * vy[bm.node(e, a)] for a in range(9)), Poly())
        Ue = sum((psi[k] * U[k][e] for k in range(na)), Poly())
        R = []
        for k in range(na):
            gx, gy = bm.ddx(psi[k]), bm.ddy(psi[k])
            R.append((Ue * (ux * gx + uy * gy)).integral() * bm.det)
        for ed in range(4):
            a0, a1 = EDGE_VERTS[ed]
            tx = corner[a1][0] - corner[a0][0]
            ty = corner[a1][1] - corner[a0][1]
            nlx, nly = ty, -tx
            xs, es = EDGE_SELF[ed]
            vn = {}
            for i, c in restrict(ux, xs, es).items():
                vn[i] = vn.get(i, Fr(0)) + c * nlx
            for i, c in restrict(uy, xs, es).items():
                vn[i] = vn.get(i, Fr(0)) + c * nly
            sign = upoly_at(vn, Fr(1, 2))
            fx, fy = ex + EDGE_NB_OFFSET[ed][0], ey + EDGE_NB_OFFSET[ed][1]
            has_nb = 0 <= fx < bm.nx and 0 <= fy < bm.ny
            if sign >= 0 or not has_nb:
                Uup = restrict(Ue, xs, es)
            else:
                f = fy * bm.nx + fx
                Uf = sum((psi[k] * U[k][f] for k in range(na)), Poly())
                xn, en = EDGE_NB[ed]
                Uup = restrict(Uf, xn, en)
            for k in range(na):
                R[k] -= upoly_int(upoly_mul(vn, Uup, restrict(psi[k], xs, es)))
        for k in range(na):
            out[k][e] = R[k] / (norms[k] * bm.det)
    return out
