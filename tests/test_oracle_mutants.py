"""The pins must discriminate: each plausible mistake planted in a copy of the
oracle source (one substitution, compiled to a scratch library on the CPU)
must make at least one pin test fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mfc_oracle.c")
PINS = [os.path.join(ROOT, "tests", f) for f in ("test_oracle_units.py", "test_oracle_scheme.py",
                                                  "test_oracle_kapila.py", "test_oracle_order.py",
                                                  "test_oracle_stretched.py", "test_oracle_cbc.py")]

MUTANTS = {
    "weno ideal weights swapped": ("dplus[3] = {0.1, 0.6, 0.3}", "dplus[3] = {0.3, 0.6, 0.1}"),
    "weno power 1 instead of 2": ("double den = (eps + beta[r]) * (eps + beta[r]);\n        ap[r] = dplus[r] / den;\n        am[r] = dminus[r] / den;\n        sp += ap[r];\n        sm += am[r];\n    }\n    double vp",
                                  "double den = (eps + beta[r]);\n        ap[r] = dplus[r] / den;\n        am[r] = dminus[r] / den;\n        sp += ap[r];\n        sm += am[r];\n    }\n    double vp"),
    "weno beta0 coefficient": ("(10.0 / 3.0) * dm1 * dm1 - (11.0 / 3.0) * dm1 * dm2", "(10.0 / 3.0) * dm1 * dm1 - (10.0 / 3.0) * dm1 * dm2"),
    "weno candidate coefficient": ("pp[1] = vi + (1.0 / 3.0) * d0", "pp[1] = vi + (1.0 / 6.0) * d0"),
    "weno mirror candidate": ("pm[2] = vi - (5.0 / 6.0) * d0 + (1.0 / 3.0) * d1", "pm[2] = vi - (5.0 / 6.0) * d0 + (1.0 / 6.0) * d1"),
    "hllc s* sign": ("double sS = (pR - pL + rhoL", "double sS = (pL - pR + rhoL"),
    "hllc Davis min": ("double sL = fmin(uL - cL, uR - cR);", "double sL = uL - cL;"),
    "hllc star energy term": ("(rho * sS + p / (sK - un))", "(rho * sS)"),
    "hllc star normal momentum": ("(m == dir ? rho * sS : rho * w[2 + m])", "(rho * w[2 + m])"),
    "hllc face alpha": ("alpha_face = w[nv - 1];", "alpha_face = wL[nv - 1];"),
    "hllc pressure on every momentum row": ("(m == dir ? p : 0.0)", "p"),
    "rhs no alpha div(u) source": ("+= h * divu[at(g, 0, i, j, k)]", "+= 0.0 * h * divu[at(g, 0, i, j, k)]"),
    "rhs source sign": ("+= h * divu[at(g, 0, i, j, k)]", "-= h * divu[at(g, 0, i, j, k)]"),
    "kapila K as printed (rho1 c2^2)": ("(z2 / alpha2 + z1 / alpha1)", "(z2 / alpha2 + rho1 * c2sq / alpha1)"),
    "kapila K sign": ("return (z2 - z1) / (z2", "return (z1 - z2) / (z2"),
    "kapila volume fractions swapped": ("(z2 / alpha2 + z1 / alpha1)", "(z2 / alpha1 + z1 / alpha2)"),
    "kapila phase sound speed without pi": ("g->gamma[0] * (p + g->pi_inf[0]) / rho1", "g->gamma[0] * p / rho1"),
    "kapila source replaces alpha1": ("h += ora_kapila_K(g, wc);", "h = ora_kapila_K(g, wc);"),
    "kapila source ignored": ("if (g->model == 1) {", "if (g->model == 7) {"),
    "weno3 ideal weights swapped": ("dplus[2] = {1.0 / 3.0, 2.0 / 3.0}", "dplus[2] = {2.0 / 3.0, 1.0 / 3.0}"),
    "weno3 candidate coefficient": ("pp[0] = (-s[0] + 3.0 * s[1]) / 2.0;", "pp[0] = (-s[0] + 2.0 * s[1]) / 2.0;"),
    "weno3 smoothness indicator": ("beta[1] = (s[2] - s[1]) * (s[2] - s[1]);", "beta[1] = (s[2] - s[0]) * (s[2] - s[1]);"),
    "weno3 mirror candidate": ("pm[1] = (3.0 * s[1] - s[2]) / 2.0;", "pm[1] = (3.0 * s[1] - s[0]) / 2.0;"),
    "weno3 weight power 1": ("double den = (eps + beta[r]) * (eps + beta[r]);\n        ap[r] = dplus[r] / den;\n        am[r] = dminus[r] / den;\n        sp += ap[r];\n        sm += am[r];\n    }\n    *at_plus",
                             "double den = (eps + beta[r]);\n        ap[r] = dplus[r] / den;\n        am[r] = dminus[r] / den;\n        sp += ap[r];\n        sm += am[r];\n    }\n    *at_plus"),
    "first order from the neighbour": ("*pl = *mi = s[2];", "*pl = *mi = s[3];"),
    "non-uniform beta second-derivative weight": ("return a1 * a1 + (13.0 / 3.0) * a2 * a2;", "return a1 * a1 + (13.0 / 12.0) * a2 * a2;"),
    "non-uniform ideal weight cell": ("cf->dplus[2] = qplus[4] / cf->plus[2][2];", "cf->dplus[2] = qplus[3] / cf->plus[2][1];"),
    "non-uniform cell average of xi^k": ("(pow(hi, k + 1) - pow(lo, k + 1)) / ((k + 1) * (hi - lo))", "(pow(hi, k + 1) - pow(lo, k + 1)) / (k + 1)"),
    "non-uniform flux difference width": ("double inv_dx = 1.0 / ora_cell_width(g, d, cell);", "double inv_dx = 1.0 / ora_cell_width(g, d, 0);"),
    "cbc incoming wave kept": ("#define ENTERS(l) (side == 0 ? (l) > 0.0 : (l) < 0.0)", "#define ENTERS(l) (side == 0 ? (l) > 1e300 : (l) < -1e300)"),
    "cbc entering test reversed": ("#define ENTERS(l) (side == 0 ? (l) > 0.0 : (l) < 0.0)", "#define ENTERS(l) (side == 0 ? (l) < 0.0 : (l) > 0.0)"),
    "cbc acoustic impedance sign": ("lam1 * (dp - rho * c * du)", "lam1 * (dp + rho * c * du)"),
    "cbc velocity rate factor": ("-(L5 - L1) / (2.0 * rho * c)", "-(L5 - L1) / (rho * c)"),
    "cbc partial density coupling": ("rkt[k] = -Lk[k] - w[k] / (rho * c2) * 0.5 * (L5 + L1);", "rkt[k] = -Lk[k];"),
    "cbc one-sided stencil": ("sg * (-3.0 * f[0] + 4.0 * f[1] - f[2]) * 0.5 * inv_dx", "sg * (-f[0] + f[1]) * inv_dx"),
    "cbc uniform stencil on non-uniform cells": ("dw[v] = cs[0] * f[0] + cs[1] * f[1] + cs[2] * f[2];",
                                                 "dw[v] = sg * (-3.0 * f[0] + 4.0 * f[1] - f[2]) * 0.5 * inv_dx;"),
    "cbc non-uniform points at faces": ("x[t] = g->faces[d] ? 0.5 * (g->faces[d][i] + g->faces[d][i + 1])",
                                        "x[t] = g->faces[d] ? g->faces[d][i]"),
    "cbc one-sided middle coefficient sign": ("c[1] = (x[0] - x[2]) /", "c[1] = (x[2] - x[0]) /"),
    "cbc energy volume-fraction term": ("((G1 - G0) * p + (P1 - P0)) * at", "((G1 - G0) * p) * at"),
    "non-uniform cfl width": ("double r = ora_cell_width(g, d, idx[d]) / (fabs(wc[2 + d]) + c);", "double r = ora_cell_width(g, d, 0) / (fabs(wc[2 + d]) + c);"),
    "rhs flux difference sign": ("(Ff[cell * nv + v] - Ff[(cell + 1) * nv + v]) * inv_dx", "(Ff[(cell + 1) * nv + v] - Ff[cell * nv + v]) * inv_dx"),
    "eos Pi without gamma": ("double h1 = g->gamma[0] * g->pi_inf[0]", "double h1 = g->pi_inf[0]"),
    "eos kinetic factor": ("ke += 0.5 * q[2 + m] * w[2 + m];", "ke += q[2 + m] * w[2 + m];"),
    "sound speed Gamma+1": ("return ((Gamma + 1.0) * p + Pi) / (Gamma * rho);", "return (Gamma * p + Pi) / (Gamma * rho);"),
    "rk3 stage-2 weights": ("0.75 * q0[t] + 0.25 * (qs[t]", "0.25 * q0[t] + 0.75 * (qs[t]"),
    "periodic ghost offset": ("int slo = g->bc[2 * d] == 1 ? n - l : 0;", "int slo = g->bc[2 * d] == 1 ? n - l + 1 : 0;"),
    "extrapolation ghost": ("int shi = g->bc[2 * d + 1] == 1 ? l - 1 : n - 1;", "int shi = g->bc[2 * d + 1] == 1 ? l - 1 : n - l;"),
    "cfl max over |u| only": ("double sd = fabs(wc[2 + d]) + c;", "double sd = fabs(wc[2 + d]);"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found exactly once: {old!r}"
    mutant_c = tmp_path / "mutant.c"
    mutant_c.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-fPIC", "-shared", "-o", str(so), str(mutant_c), "-lm"],
                   check=True)
    env = dict(os.environ, MFC_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PINS],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"no pin failed for mutant '{name}':\n{r.stdout[-2000:]}"

# Planted mistakes in the indicator oracle (Python source; a mutated copy is
# loaded as a module and the pins that take the module as an argument run on
# it).
IND_SRC = os.path.join(ROOT, "oracle", "indicator.py")
IND_MUTANTS = {
    "adam without bias correction": ("mhat = m / (1.0 - b1 ** t)\n        vhat = v / (1.0 - b2 ** t)",
                                     "mhat = m\n        vhat = v"),
    "adam |g| in the second moment": ("(1.0 - b2) * grads[k] ** 2", "(1.0 - b2) * np.abs(grads[k])"),
    "adam eps inside the square root": ("(np.sqrt(vhat) + eps)", "np.sqrt(vhat + eps)"),
    "adam first moment decay": ("m[...] = b1 * m + (1.0 - b1) * grads[k]", "m[...] = b2 * m + (1.0 - b2) * grads[k]"),
}


@pytest.mark.parametrize("name", sorted(IND_MUTANTS))
def test_indicator_pins_catch_planted_mistake(name):
    import importlib.util
    import test_oracle_adam as pins
    old, new = IND_MUTANTS[name]
    src = open(IND_SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found exactly once: {old!r}"
    spec = importlib.util.spec_from_loader("indicator_mutant", loader=None)
    mod = importlib.util.module_from_spec(spec)
    exec(compile(src.replace(old, new), "indicator_mutant.py", "exec"), mod.__dict__)
    caught = 0
    for check in (pins.check_first_step_closed_form, pins.check_matches_torch):
        try:
            check(mod)
        except AssertionError:
            caught += 1
    assert caught > 0, f"no Adam pin failed for mutant '{name}'"
