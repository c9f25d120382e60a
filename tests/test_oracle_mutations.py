"""Planted mistakes in the oracle, on the CPU: each mutation below is a
plausible error (a dropped term, a wrong sign or index, a swapped operand or
exponent) applied to a copy of oracle/hfav_oracle.c; the copy is compiled
and the oracle's pins are run against it.  Every mutant must fail at least
one pin, which shows the pins are strong enough to catch that kind of
mistake anywhere in the oracle."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "hfav_oracle.c")

HDIFF, EULER, L7, MLP = ("test_oracle_hdiff.py", "test_oracle_euler.py", "test_oracle_biharm_chain.py",
                         "test_oracle_biharm_chain.py")
NORM = "test_oracle_norm.py"

# (name, original text, mutated text, pin file)
MUTANTS = [
    ("hdiff Laplacian centre weight", "- 4.0 * PAD(k, j, i)", "- 3.0 * PAD(k, j, i)", HDIFF),
    ("hdiff x limiter inverted", "if (limiter && f * (PAD(k, j, i + 1) - PAD(k, j, i)) > 0.0) f = 0.0;",
     "if (limiter && f * (PAD(k, j, i + 1) - PAD(k, j, i)) < 0.0) f = 0.0;", HDIFF),
    ("hdiff y flux difference sign", "(FLY(k, j, i) - FLY(k, j - 1, i))", "(FLY(k, j, i) + FLY(k, j - 1, i))", HDIFF),
    ("hdiff y flux index", "double f = LAP(k, j + 1, i) - LAP(k, j, i);",
     "double f = LAP(k, j + 1, i) - LAP(k, j - 1, i);", HDIFF),
    ("shock derivative sign", "*fd = q * (1.0 - (p - pk) / (2.0 * (B + p)));",
     "*fd = q * (1.0 + (p - pk) / (2.0 * (B + p)));", EULER),
    ("shock constant B inverted", "double B = (g - 1.0) / (g + 1.0) * pk;",
     "double B = (g + 1.0) / (g - 1.0) * pk;", EULER),
    ("rarefaction exponent", "pow(pr, (g - 1.0) / (2.0 * g))", "pow(pr, (g + 1.0) / (2.0 * g))", EULER),
    ("star velocity sign", "*us = 0.5 * (ul + ur) + 0.5 * (fr - fl);", "*us = 0.5 * (ul + ur) + 0.5 * (fl - fr);",
     EULER),
    ("left shock speed sign", "double sl = ul - cl * sqrt(g2 * pml + g1);",
     "double sl = ul + cl * sqrt(g2 * pml + g1);", EULER),
    ("left fan velocity", "W[1] = g5 * (cl + g7 * ul);", "W[1] = g5 * (cl - g7 * ul);", EULER),
    ("left shock density", "W[0] = rl * (pml + g6) / (pml * g6 + 1.0);",
     "W[0] = rl * (pml - g6) / (pml * g6 + 1.0);", EULER),
    ("right fan density exponent", "W[0] = rr * pow(c, g4);", "W[0] = rr * pow(c, g3);", EULER),
    ("van Leer factor 2", "2.0 * a * b / (a + b)", "a * b / (a + b)", EULER),
    ("trace velocity sign", "LA(Wm, 1, l, m) = un + (c / r) * (cp[3] - cp[0]);",
     "LA(Wm, 1, l, m) = un + (c / r) * (cp[0] - cp[3]);", EULER),
    ("entropy wave strength", "dr - dp / (c * c),", "dr + dp / (c * c),", EULER),
    ("trace half-step sign", "cp[w] = lam[w] >= 0.0 ? 0.5 * (1.0 - nu * lam[w]) * alp[w] : 0.0;",
     "cp[w] = lam[w] >= 0.0 ? 0.5 * (1.0 + nu * lam[w]) * alp[w] : 0.0;", EULER),
    ("momentum flux pressure sign", "LA(Fx, 1, l, m) = r * un * un + p;", "LA(Fx, 1, l, m) = r * un * un - p;",
     EULER),
    ("energy flux drops p", "LA(Fx, 3, l, m) = un * (et + p);", "LA(Fx, 3, l, m) = un * et;", EULER),
    ("update flux index", "U[0 * plane + s] = LA(Ug, 0, l, m) - nu * (LA(Fx, 0, l, m) - LA(Fx, 0, l, m - 1));",
     "U[0 * plane + s] = LA(Ug, 0, l, m) - nu * (LA(Fx, 0, l, m + 1) - LA(Fx, 0, l, m));", EULER),
    ("y sweep momentum roles", "const int fn = dir == 0 ? 1 : 2, ft = dir == 0 ? 2 : 1;",
     "const int fn = 1, ft = 2;", EULER),
    ("CFL speed ignores v", "double a = fabs(u) + c, b = fabs(v) + c;", "double a = fabs(u) + c, b = fabs(u) + c;",
     EULER),
    ("EOS drops transverse kinetic energy", "double p = (g - 1.0) * (e - 0.5 * r * (un * un + ut * ut));",
     "double p = (g - 1.0) * (e - 0.5 * r * (un * un));", EULER),
    ("7-point centre weight", "- 6.0 * U3(k, j, i);", "- 5.0 * U3(k, j, i);", L7),
    ("7-point z neighbour", "(U3(k + 1, j, i) + U3(k - 1, j, i))", "(U3(k + 1, j, i) + U3(k + 1, j, i))", L7),
    ("biharmonic update sign", "out[q] = cur[q] - nu * l2[q];", "out[q] = cur[q] + nu * l2[q];", L7),
    ("linear chain mirrored offset", "int ii = wrap(i + op[3 * q], nx)", "int ii = wrap(i - op[3 * q], nx)", L7),
    ("linear chain transposed coefficients", "acc += cp[((size_t)o * fi + f) * no + q] *",
     "acc += cp[((size_t)f * fo + o) * no + q] *", L7),
    ("MLP loss gradient factor 2", "double dy = 2.0 * r / n;", "double dy = r / n;", MLP),
    ("MLP layer-3 weight gradient activation", "gW3[(size_t)o * H + i] += d3[o] * h2[i];",
     "gW3[(size_t)o * H + i] += d3[o] * h1[i];", MLP),
    ("Adam drops bias correction", "double mh = m[q] / c1, vh = v[q] / c2;", "double mh = m[q], vh = v[q] / c2;",
     MLP),
    ("normalisation flux index", "(periodic ? wrap(i + 1, ni) : clampi(i + 1, ni))",
     "(periodic ? wrap(i + 2, ni) : clampi(i + 1, ni))", NORM),
    ("normalisation transmissive end wraps", "(periodic ? wrap(i + 1, ni) : clampi(i + 1, ni))",
     "(periodic ? wrap(i + 1, ni) : wrap(i + 1, ni))", NORM),
    ("normalisation square dropped", "acc += v * v;", "acc += v;", NORM),
    ("normalisation root dropped", "for (int j = 0; j < nj; ++j) nn[j] = sqrt(sn[j]);",
     "for (int j = 0; j < nj; ++j) nn[j] = sn[j];", NORM),
    ("normalisation update sign", "out[o] = u[o] - c * d[o];", "out[o] = u[o] + c * d[o];", NORM),
]


def _run_mutant(args):
    name, old, new, pins, workdir = args
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {name}"
    d = os.path.join(workdir, "m%d" % abs(hash(name)))
    os.makedirs(d, exist_ok=True)
    cpath = os.path.join(d, "m.c")
    with open(cpath, "w") as f:
        f.write(src.replace(old, new))
    lib = os.path.join(d, "liboracle_mutant.so")
    subprocess.run(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-std=c11", "-shared",
                    "-fPIC", cpath, "-o", lib, "-lm"], check=True, capture_output=True)
    env = dict(os.environ, HFAV_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(HERE, pins)], cwd=ROOT, env=env, capture_output=True, text=True)
    return name, r.returncode


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc to build the mutants")
def test_every_planted_mistake_fails_a_pin(tmp_path):
    jobs = [(n, o, m, p, str(tmp_path)) for n, o, m, p in MUTANTS]
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(_run_mutant, jobs))
    missed = [n for n, rc in results if rc == 0]
    assert not missed, f"mutants that pass every pin: {missed}"
