"""Plausible mistakes planted in the oracle are caught by its pins.

Each mutant below is the oracle's C source with one textual change of the
kind the pins are meant to exclude (a dropped term, a wrong sign, a wrong
index or weight, a wrong time level).  The mutant is compiled with the
oracle's own flags and the pin suite (the ``test_oracle_*`` and
``test_golden`` files, fastest first, stopping at the first failure) is run
against it in a subprocess; every mutant must make at least one pin fail.
The unmutated source, compiled the same way, must pass the whole suite.
Mutants that leave the scheme's results unchanged (reordering an exact sum,
renumbering velocities) are not mistakes and are not listed.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbem_oracle.c")

# the pin files, fastest first
PINS = ["tests/test_oracle_identities.py", "tests/test_golden.py", "tests/test_oracle_boundaries.py",
        "tests/test_oracle_anisotropy.py", "tests/test_oracle_dispersion_ade.py",
        "tests/test_oracle_physics.py"]

# (name, original text, planted mistake); the original occurs exactly once
MUTANTS = [
    ("moving weight (1-w0)/D instead of (1-w0)/(2D)",
     "return i == 0 ? w0 : (1.0 - w0) / (2.0 * D);", "return i == 0 ? w0 : (1.0 - w0) / (double)D;"),
    ("equilibrium wedge with + instead of -",
     "double wedge = c[i][a] * Bbar[b] - c[i][b] * Bbar[a];",
     "double wedge = c[i][a] * Bbar[b] + c[i][b] * Bbar[a];"),
    ("Bbar = K (no division by the first moments' multiplicity)",
     "Bbar[b] = K[b] / rs;", "Bbar[b] = K[b];"),
    ("Bbar denominator summed over all axes",
     "if (a != b) rs += 2.0 * w[1 + a] / cl2;", "rs += 2.0 * w[1 + a] / cl2;"),
    ("equilibrium prefactor w_i instead of w_i/c^2",
     "double wc = w[i] / cl2;\n        for (int a = 0; a < D; ++a)\n            for (int b = 0; b < D; ++b) {\n"
     "                double wedge",
     "double wc = w[i];\n        for (int a = 0; a < D; ++a)\n            for (int b = 0; b < D; ++b) {\n"
     "                double wedge"),
    ("first moment with c_ib instead of c_ia",
     "s += c[i][a] * gc[(i * D + a) * D + b];", "s += c[i][b] * gc[(i * D + a) * D + b];"),
    ("zeroth moment drops the rest particle",
     "for (int i = 0; i < Q; ++i) s += gc[(i * D + a) * D + b];",
     "for (int i = 1; i < Q; ++i) s += gc[(i * D + a) * D + b];"),
    ("E recovered with the wrong sign", "E[gm] = -0.5 * s;", "E[gm] = 0.5 * s;"),
    ("initial Lambda with the wrong sign", "Lam[a * D + b] = -s;", "Lam[a * D + b] = s;"),
    ("Levi-Civita: one cyclic permutation taken as odd",
     "(a == 2 && b == 0 && c == 1))", "(a == 2 && b == 1 && c == 0))"),
    ("collision rate tau instead of 1/tau", "double om = 1.0 / tau;", "double om = tau;"),
    ("source tensor with the wrong sign", "double T = -wc * es;", "double T = wc * es;"),
    ("source tensor without the w_i/c^2 weight", "double T = -wc * es;", "double T = -es;"),
    ("streaming against the velocity",
     "long xd = neighbour(o, x, o->c[i], +1);", "long xd = neighbour(o, x, o->c[i], -1);"),
    ("periodic wrap off by one below zero",
     "static long wrap(long v, long n) { v %= n; return v < 0 ? v + n : v; }",
     "static long wrap(long v, long n) { v %= n; return v < 0 ? v + n - 1 : v; }"),
    ("c_L^2 with D-1 in place of D",
     "double cl2 = (1.0 - o->w0_vac) / ((double)D * e * m);",
     "double cl2 = (1.0 - o->w0_vac) / ((double)(D - 1) * e * m);"),
    ("rest weight 1 - (D-1) c_L^2", "double w0 = 1.0 - D * cl2;", "double w0 = 1.0 - (D - 1) * cl2;"),
    ("vacuum speed without the D-1",
     "double cvac2 = (1.0 - o->w0_vac) / (double)(D * (D - 1));",
     "double cvac2 = (1.0 - o->w0_vac) / (double)D;"),
    ("grad ln mu with the wrong sign",
     "0.5 * (log(o->mu_r[xp]) - log(o->mu_r[xm]))", "0.5 * (log(o->mu_r[xm]) - log(o->mu_r[xp]))"),
    ("mu term with c_L^2 in place of c_M^2",
     "double cM2 = o->cL2[x] / (double)(D - 1);", "double cM2 = o->cL2[x];"),
    ("mu term with the wrong sign",
     "S[gm] = cM2 * mu_term - a * o->jd[gm * n + x] / o->eps_abs[x];",
     "S[gm] = -cM2 * mu_term - a * o->jd[gm * n + x] / o->eps_abs[x];"),
    ("current of the next step (source time level)",
     "double a = amp ? amp[s] : 0.0;", "double a = amp ? amp[s + 1 < nsteps ? s + 1 : s] : 0.0;"),
    ("current divided by eps_r instead of eps_abs",
     "- a * o->jd[gm * n + x] / o->eps_abs[x];", "- a * o->jd[gm * n + x] / (o->eps_abs[x] * o->cL2[x]);"),
    ("dispersion: restoring term with the wrong sign", "- w02 * Po) / (1.0 + 0.5 * gam);",
     "+ w02 * Po) / (1.0 + 0.5 * gam);"),
    ("dispersion: damping not halved", "double Jn = ((1.0 - 0.5 * gam) * Jo",
     "double Jn = ((1.0 - gam) * Jo"),
    ("dispersion: polarisation source with the wrong sign", "out[a2 * D + b2] += -es / o->cL2[x];",
     "out[a2 * D + b2] += es / o->cL2[x];"),
    ("dispersion: P advanced with the old J", "o->pol[gm * n + x] = Po + Jn;", "o->pol[gm * n + x] = Po + Jo;"),
    ("absorber applied to the rest particle only", "for (int k = 0; k < Q * D * D; ++k) out[k] *= o->keep[x];",
     "for (int k = 0; k < D * D; ++k) out[k] *= o->keep[x];"),
    ("absorber keeps sigma instead of 1 - sigma", "o->keep[x] = 1.0 - sigma[x];", "o->keep[x] = sigma[x];"),
    ("PEC and PMC walls swapped", "double flip = o->bc[wall] == 1 ? -1.0 : 1.0;",
     "double flip = o->bc[wall] == 1 ? 1.0 : -1.0;"),
    ("wall reflection: both indices normal", "double sg = (a == wall || b == wall) ? flip : -flip;",
     "double sg = (a == wall && b == wall) ? flip : -flip;"),
    ("wall: re-enters along the same velocity", "if (o->c[j][wall] == -o->c[i][wall]) io = j;",
     "if (o->c[j][wall] == o->c[i][wall]) io = j;"),
    ("wall medium: periodic neighbour for the ln mu gradient",
     "if (o->bc[k] != 0 && (w < 0 || w >= nn[k])) w = v[k];", "(void)0;"),
    ("anisotropy: moving weight s_a instead of s_a/2", "wax[a * n + x] = 0.5 * sa;", "wax[a * n + x] = sa;"),
    ("anisotropy: c^2 the sum instead of the mean", "o->cL2[x] = sum / (double)D;", "o->cL2[x] = sum;"),
    ("anisotropy: eps_abs left isotropic",
     "o->eps_abs[x] = (double)(D - 1) / (o->mu_r[x] * o->cL2[x]);", "(void)0;"),
    ("Q_c weighted by w_i instead of 1/w_i", "q += s / w;", "q += s * w;"),
    ("energy: B^2 times mu_r", "en += o->eps_abs[x] * e2 + b2 / o->mu_r[x];",
     "en += o->eps_abs[x] * e2 + b2 * o->mu_r[x];"),
    ("div B: difference not halved",
     "d += 0.5 * (Bf[k * n + neighbour(o, x, dd, +1)] - Bf[k * n + neighbour(o, x, dd, -1)]);",
     "d += (Bf[k * n + neighbour(o, x, dd, +1)] - Bf[k * n + neighbour(o, x, dd, -1)]);"),
    ("reported B = Bbar instead of K", "for (int b = 0; b < D; ++b) B[b] = K[b];",
     "for (int b = 0; b < D; ++b) B[b] = K[b] / (D - 1);"),
    ("initial Bbar = B (no division)", "bbar_of(D, w, o->cL2[x], Bp, Bbar);",
     "for (int b = 0; b < D; ++b) Bbar[b] = Bp[b];"),
    ("Q_c without the c_L^2 factor", "qc += o->cL2[x] * q;", "qc += q;"),
    ("energy without eps_abs", "en += o->eps_abs[x] * e2 + b2 / o->mu_r[x];", "en += e2 + b2 / o->mu_r[x];"),
    ("anisotropy: rest weight 1 - sum/2", "o->w0[x] = 1.0 - sum;", "o->w0[x] = 1.0 - 0.5 * sum;"),
    ("anisotropy: weights of the next axis", "if (o->c[i][a] != 0) w[i] = o->wax[a * o->n + x];",
     "if (o->c[i][a] != 0) w[i] = o->wax[((a + 1) % o->D) * o->n + x];"),
    ("Bbar denominator without the factor 2", "if (a != b) rs += 2.0 * w[1 + a] / cl2;",
     "if (a != b) rs += w[1 + a] / cl2;"),
    ("dispersion: source from the old J", "Sp[gm] = -Jn;", "Sp[gm] = -Jo;"),
    ("dispersion: damping denominator 1 + gamma", "wp2 * E[gm] - w02 * Po) / (1.0 + 0.5 * gam);",
     "wp2 * E[gm] - w02 * Po) / (1.0 + gam);"),
    ("wall test off by one at the low face", "(v[a] + o->c[i][a] < 0 || v[a] + o->c[i][a] >= nn[a])",
     "(v[a] + o->c[i][a] <= 0 || v[a] + o->c[i][a] >= nn[a])"),
    ("source footprint overwritten instead of summed", "o->jd[comp[k] * o->n + cell[k]] += weight[k];",
     "o->jd[comp[k] * o->n + cell[k]] = weight[k];"),
    ("initial fields: B used as K in 3D (no Bbar)", "double w[7], Bp[3] = {B[x], B[n + x], B[2 * n + x]};",
     "double w[7], Bp[3] = {B[x] * (D - 1), B[n + x] * (D - 1), B[2 * n + x] * (D - 1)};"),
]


def compile_variant(text: str, path: str) -> None:
    src = path[:-3] + ".c"
    with open(src, "w") as f:
        f.write(text)
    subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable", src,
                    "-o", path, "-lm"], check=True, capture_output=True)


def run_pins(lib: str, stop_first: bool) -> subprocess.CompletedProcess:
    env = dict(os.environ, LBEM_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu"]
    if stop_first:
        cmd.append("-x")
    return subprocess.run(cmd + PINS, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)


def check_mutant(k: int, tmp: str):
    name, old, new = MUTANTS[k]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutant {k} ({name}): original text found {text.count(old)} times"
    lib = os.path.join(tmp, f"mutant{k}.so")
    compile_variant(text.replace(old, new), lib)
    r = run_pins(lib, stop_first=True)
    failed = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
    return k, r.returncode, failed[:1]


def test_unmutated_source_passes_the_pins(tmp_path):
    lib = str(tmp_path / "control.so")
    compile_variant(open(SRC).read(), lib)
    r = run_pins(lib, stop_first=False)
    assert r.returncode == 0, r.stdout[-3000:]


def test_every_planted_mistake_fails_a_pin(tmp_path):
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(lambda k: check_mutant(k, str(tmp_path)), range(len(MUTANTS))))
    survivors = [MUTANTS[k][0] for k, rc, _ in results if rc == 0]
    for k, rc, failed in results:
        print(f"{MUTANTS[k][0]}: {'caught by ' + failed[0][7:] if failed else 'rc=%d' % rc}")
    assert not survivors, survivors


@pytest.mark.parametrize("k", range(len(MUTANTS)))
def test_mutant_text_is_present(k):
    assert open(SRC).read().count(MUTANTS[k][1]) == 1, MUTANTS[k][0]
