"""Mutation check of the oracle's pins.

Each mutant below is one plausible mistake planted in a copy of the oracle's
C source (a dropped factor, a flipped sign, a swapped index or component, a
wrong order of the phases). The copy is compiled with the oracle's own flags
into a temporary library, the oracle pin tests are run against it in a
subprocess (``oracle.ENV_LIB`` selects the library), and the test asserts that
at least one pin fails. A mutant that every pin accepts means a part of the
oracle that nothing independent of it checks.

Mistakes are planted on the CPU only, in temporary copies; the committed
oracle is never modified.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mevp_oracle.c")
PIN_FILES = ["tests/test_oracle_tables.py", "tests/test_oracle_pins.py",
             "tests/test_oracle_composition.py", "tests/test_brute_2x2.py",
             "tests/test_oracle_iso.py", "tests/test_oracle_advection.py"]

# name -> [(text in the oracle source, replacement), ...]; each text occurs once
MUTANTS = {
    # velocity update
    "force sign in the velocity update": [("+ d * ox + F[j];", "+ d * ox - F[j];")],
    "force components swapped": [("+ d * ox + F[j];", "+ d * ox + F[nn + j];"),
                                 ("+ d * oy + F[nn + j];", "+ d * oy + F[j];")],
    "Coriolis sign": [("double b = p->f_cor * MH[j];", "double b = -p->f_cor * MH[j];")],
    "beta term dropped from the diagonal": [("double a = c * (1.0 + p->beta) + d;",
                                            "double a = c * p->beta + d;")],
    "ocean drag not implicit": [("double a = c * (1.0 + p->beta) + d;",
                                 "double a = c * (1.0 + p->beta);")],
    "ocean drag x1.01": [("double d = mA[j] * p->rho_o", "double d = 1.01 * mA[j] * p->rho_o")],
    "ocean drag magnitude without the ice velocity": [
        ("sqrt((ox - vx) * (ox - vx) + (oy - vy) * (oy - vy))", "sqrt(ox * ox + oy * oy)")],
    "air stress weighted by the ice mass": [("+ mA[j] * tau[j] +", "+ MH[j] * tau[j] +")],
    "v^n replaced by v^(p-1)": [("c * (p->beta * vx + vn[j])", "c * (p->beta * vx + vx)")],
    "top boundary not held at rest": [("if (ix == 0 || iy == 0 || ix == NX - 1 || iy == NY - 1) {",
                                       "if (ix == 0 || iy == 0 || ix == NX - 1) {")],
    "air stress component": [("tau[nn + j] = p->rho_a * p->C_a * sp * uy;",
                              "tau[nn + j] = p->rho_a * p->C_a * sp * ux;")],
    # subcycle order
    "divergence from the old stress": [(
        "    or_strain(m, v, E);                                /* sigma^(p) from v^(p-1) ... */\n"
        "    or_stress(m, p, E, H, A, S);\n"
        "    or_divergence(m, S, F);",
        "    or_divergence(m, S, F);\n    or_strain(m, v, E);\n    or_stress(m, p, E, H, A, S);")],
    # stress update
    "s11 and s22 swapped in the projection": [("      project(m, e, sg[c], pc);",
                                               "      project(m, e, sg[2 - c], pc);")],
    "e11 and e22 swapped into the point law": [(
        "      vp_stress_point(p, h, a, e11, e12, e22, sq, NULL, NULL);",
        "      vp_stress_point(p, h, a, e22, e12, e11, sq, NULL, NULL);")],
    "relaxation skips the last coefficient": [("      for (int k = 0; k < ns; ++k) {\n        double *Sk",
                                               "      for (int k = 0; k < ns - 1; ++k) {\n        double *Sk")],
    "relaxation weight of the other form": [("ainv = 1.0 / p->alpha;", "ainv = 1.0 / (p->alpha + 1.0);")],
    "5/8 and 3/8 swapped": [("s[0] = PD * (5.0 / 8.0 * e11 + 3.0 / 8.0 * e22) - 0.5 * P;",
                             "s[0] = PD * (3.0 / 8.0 * e11 + 5.0 / 8.0 * e22) - 0.5 * P;")],
    "shear factor 1/2 for 1/4": [("s[1] = PD * (1.0 / 4.0) * e12;", "s[1] = PD * (1.0 / 2.0) * e12;")],
    "Delta cross term sign": [("+ 1.5 * e11 * e22 +", "- 1.5 * e11 * e22 +")],
    "ice strength exp(-C a)": [("exp(-p->C * (1.0 - a));", "exp(-p->C * a);")],
    "concentration clamp at one dropped": [("*a = fmin(1.0, fmax(0.0, as));", "*a = fmax(0.0, as);")],
    "higher concentration coefficients ignored": [("as += A[k * ne + e] * m->psiA[k][q];",
                                                   "as += A[k * ne + e] * m->psiA[0][q];")],
    # strain
    "strain 1/2 dropped": [("= 0.5 * (dvxdy + dvydx);", "= (dvxdy + dvydx);")],
    "strain gradient component": [("dvxdy += vx[a] * gy[a * ng + q];", "dvxdy += vx[a] * gx[a * ng + q];")],
    # divergence
    "divergence sign": [("fe[e * 18 + a] = -fx;", "fe[e * 18 + a] = fx;")],
    "divergence y row x(1+1e-10)": [("fe[e * 18 + 9 + a] = -fy;", "fe[e * 18 + 9 + a] = -fy * (1.0 + 1e-10);")],
    "divergence y row uses s11": [("fy += wd[q] * (s12[q] * gx[a * ng + q] + s22[q] * gy[a * ng + q]);",
                                   "fy += wd[q] * (s11[q] * gx[a * ng + q] + s22[q] * gy[a * ng + q]);")],
    "divergence x row gradients swapped": [(
        "fx += wd[q] * (s11[q] * gx[a * ng + q] + s12[q] * gy[a * ng + q]);",
        "fx += wd[q] * (s11[q] * gy[a * ng + q] + s12[q] * gx[a * ng + q]);")],
    # masses
    "concentration mass without the basis function": [("sa += wd[q] * c * m->phi[a][q];",
                                                       "sa += wd[q] * c / 9.0;")],
    "ice mass without rho_i": [("sh += wd[q] * p->rho_i * h * m->phi[a][q];",
                                "sh += wd[q] * h * m->phi[a][q];")],
    # reference element, geometry, projection
    "Gauss weight": [("w[1] = 4.0 / 9.0;", "w[1] = 4.0 / 9.5;")],
    "DG basis constant": [("case 3: return s * s - 1.0 / 12.0;", "case 3: return s * s - 1.0 / 6.0;")],
    "Lagrange derivative": [("if (i == 1) return 4.0 - 8.0 * t;", "if (i == 1) return 4.0 - 4.0 * t;")],
    "local node order transposed": [("return node_index(m, 2 * ex + c, 2 * ey + b);",
                                     "return node_index(m, 2 * ex + b, 2 * ey + c);")],
    "bilinear Jacobian entry": [("J[3] = (1.0 - xi) * (Y[2] - Y[0]) + xi * (Y[3] - Y[1]);",
                                 "J[3] = (1.0 - eta) * (Y[2] - Y[0]) + eta * (Y[3] - Y[1]);")],
    "isoparametric Jacobian entry": [("J[1] += (m->nx_[j] - x0) * dy;", "J[1] += (m->nx_[j] - x0) * dx;")],
    "mass matrix symmetric part only": [(
        "for (int q = 0; q < m->ng; ++q) s += m->psiS[k][q] * wd[q] * m->psiS[l][q];",
        "for (int q = 0; q < m->ng; ++q) s += m->psiS[k][q] * wd[q] * m->psiS[k][q];")],
    "projection without the weights": [("s += m->psiS[k][q] * wd[q] * g[q];", "s += m->psiS[k][q] * g[q];")],
    "transposed Cholesky back substitution": [(
        "for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * x[k];",
        "for (int k = i + 1; k < n; ++k) s -= L[i * n + k] * x[k];")],
    # advection
    "advection upwind side": [("if (vn >= 0.0 || !has_nb) {", "if (vn <= 0.0 || !has_nb) {")],
    "advection edge normal sign": [("double nlx = ty, nly = -tx;", "double nlx = -ty, nly = tx;")],
    "advection volume term sign": [("R[k] += w * det * Uq * (ux * gx + uy * gy);",
                                    "R[k] -= w * det * Uq * (ux * gx + uy * gy);")],
    "advection second RK blend": [("U2[i] = 0.75 * U[i] + 0.25 * (U1[i] + dt * L[i]);",
                                   "U2[i] = 0.5 * U[i] + 0.5 * (U1[i] + dt * L[i]);")],
    "advection final RK stage input": [("U[i] = U[i] / 3.0 + 2.0 / 3.0 * (U2[i] + dt * L[i]);",
                                        "U[i] = U[i] / 3.0 + 2.0 / 3.0 * (U1[i] + dt * L[i]);")],
    "advection neighbour trace point": [("case 0: *xi = u; *eta = 1.0; return;",
                                         "case 0: *xi = 1.0 - u; *eta = 1.0; return;")],
    "advection edge weight": [("R[k] -= gw[g] * vn * Uup * dg_basis(k, xi, eta);",
                               "R[k] -= gw[1] * vn * Uup * dg_basis(k, xi, eta);")],
    "advection basis derivative": [("case 4: *dxi = t; *deta = s; return;",
                                    "case 4: *dxi = s; *deta = t; return;")],
    "advection gradient x row J10 sign": [("double gx = (J11 * dxi - J10 * deta) / det;",
                                           "double gx = (J11 * dxi + J10 * deta) / det;")],
    "advection gradient y row J01 sign": [("double gy = (-J01 * dxi + J00 * deta) / det;",
                                           "double gy = (J01 * dxi + J00 * deta) / det;")],
    "reference xi-gradient table with xi and eta swapped": [
        ("if (dxi) dxi[a * ng + q] = dlag2(c, xi) * lag2(b, eta);",
         "if (dxi) dxi[a * ng + q] = dlag2(c, eta) * lag2(b, xi);")],
    "reference eta-gradient table differentiates in xi": [
        ("if (deta) deta[a * ng + q] = lag2(c, xi) * dlag2(b, eta);",
         "if (deta) deta[a * ng + q] = dlag2(c, xi) * lag2(b, eta);")],
    # degenerate and edge cases, accessors
    "ice-free node keeps its y velocity": [("      v[nn + j] = 0.0;\n    } else {", "    } else {")],
    "concentration not advected": [("  advect_field(m, dt, v, A);\n", "")],
    "zero subcycles rejected": [("if (!m || !p || n_sub < 0) return -1;",
                                 "if (!m || !p || n_sub <= 0) return -1;")],
    "geometry accessor copies part of the y gradients": [
        ("memcpy(dphiy, m->dphiy + (size_t)e * 9 * ng, sizeof(double) * 9 * ng);",
         "memcpy(dphiy, m->dphiy + (size_t)e * 9 * ng, sizeof(double) * 8 * ng);")],
}


def _mutated_source(edits):
    text = open(SRC).read()
    for old, new in edits:
        n = text.count(old)
        assert n == 1, f"mutation text occurs {n} times: {old!r}"
        text = text.replace(old, new)
    return text


def _run_mutant(name, edits, workdir):
    import oracle.build as ob
    tag = "".join(ch if ch.isalnum() else "_" for ch in name)
    src = os.path.join(workdir, f"{tag}.c")
    lib = os.path.join(workdir, f"lib{tag}.so")
    with open(src, "w") as f:
        f.write(_mutated_source(edits))
    ob.build(src=src, lib=lib)
    env = dict(os.environ, MEVP_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu"] + PIN_FILES, cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    return name, r.returncode, r.stdout[-2000:]


def test_every_planted_mistake_fails_a_pin():
    # the mutation texts still match the source (else the test would check nothing)
    for name, edits in MUTANTS.items():
        _mutated_source(edits)
    workdir = tempfile.mkdtemp(prefix="mevp_mutants_")
    try:
        workers = max(1, min(8, os.cpu_count() or 1))
        with ThreadPoolExecutor(workers) as ex:
            results = list(ex.map(lambda kv: _run_mutant(kv[0], kv[1], workdir), MUTANTS.items()))
    finally:
        shutil.rmtree(workdir, ignore_errors=True)
    survivors = []
    for name, rc, out in results:
        # rc 1: some test failed; anything else (collection error, crash) is not a pin failing
        if rc != 1 or " failed" not in out:
            survivors.append((name, rc, out.splitlines()[-1:] if out else ""))
    assert not survivors, survivors


@pytest.mark.parametrize("name", ["divergence from the old stress"])
def test_mutation_texts_apply_once(name):
    assert _mutated_source(MUTANTS[name]) != open(SRC).read()
