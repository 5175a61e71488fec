"""The oracle pins catch planted mistakes (CPU).

Each case plants one plausible mistake in a copy of the oracle's C source (a
dropped term, a wrong sign, index or constant, a transposed operand), builds
it, and runs the pin suite against it through GFMC_ORACLE_LIB: some pin must
fail.  The oracle itself is never changed; the copies live in a temporary
directory.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "gfmc_oracle.c")

# (name, text in the oracle, replacement)
MUTANTS = [
    ("philox Weyl constant", "W1 = 0xBB67AE8584CAA73BULL", "W1 = 0xBB67AE8584CAA73CULL"),
    ("uniform draw resolution", "(double)(r >> 11) * 0x1.0p-53", "(double)(r >> 12) * 0x1.0p-52"),
    ("site index map", "return (int64_t)(uint64_t)(p >> 64);", "return (int64_t)(uint64_t)(p >> 63);"),
    ("neighbour +x step", "case 0: x = (x + 1) % L; break;", "case 0: x = (x + 2) % L; break;"),
    ("hopping: conjugated", "out[1] = cos(0.5 * (th_i + th_j)) * sin(0.5 * (ph_i - ph_j));",
     "out[1] = -cos(0.5 * (th_i + th_j)) * sin(0.5 * (ph_i - ph_j));"),
    ("hopping: theta difference in the phase term",
     "out[1] = cos(0.5 * (th_i + th_j)) * sin(0.5 * (ph_i - ph_j));",
     "out[1] = cos(0.5 * (th_i - th_j)) * sin(0.5 * (ph_i - ph_j));"),
    ("hopping: scale t dropped", "val[6 * i + d] = -(p->t / p->a) * hop(",
     "val[6 * i + d] = -(1.0 / p->a) * hop("),
    ("recursion: sign of the a_{n-2} term", "next[i] = 2.0 * next[i] - prev[i];",
     "next[i] = 2.0 * next[i] + prev[i];"),
    ("bond change sign", "cplx dd = h_new - h_old;", "cplx dd = h_old - h_new;"),
    ("contraction: conjugate dropped", "vv += conj(dl[j]) * dl[k] * m[1 + j][1 + k];",
     "vv += dl[j] * dl[k] * m[1 + j][1 + k];"),
    ("contraction: transposed ov", "ov += dl[k] * m[0][1 + k];", "ov += dl[k] * m[1 + k][0];"),
    ("Jackson coefficient", "g[n] = ((M - n + 1.0) * cos(q * n)", "g[n] = ((M - n) * cos(q * n)"),
    ("Lorentz coefficient", "g[n] = sinh(lambda * (1.0 - (double)n / M)) / sinh(lambda);",
     "g[n] = sinh(lambda * (1.0 - (double)n / M));"),
    ("Lorentz coefficient: M + 1 in the ratio", "g[n] = sinh(lambda * (1.0 - (double)n / M)) / sinh(lambda);",
     "g[n] = sinh(lambda * (1.0 - (double)n / (M + 1))) / sinh(lambda);"),
    ("Lorentz coefficient: cosh", "g[n] = sinh(lambda * (1.0 - (double)n / M)) / sinh(lambda);",
     "g[n] = cosh(lambda * (1.0 - (double)n / M)) / cosh(lambda);"),
    ("Lorentz coefficient: shifted index", "g[n] = sinh(lambda * (1.0 - (double)n / M)) / sinh(lambda);",
     "g[n] = sinh(lambda * (1.0 - (double)(n + 1) / M)) / sinh(lambda);"),
    ("green: mu_0 not halved", "if (n == 0) m *= 0.5;", "if (n == 0) m *= 1.0;"),
    ("green: node offset", "double thk = PI * (k + 0.5) / K;\n    cplx s = 0;",
     "double thk = PI * (k + 1.0) / K;\n    cplx s = 0;"),
    ("determinant: G not rescaled by a", "cplx goo = (Goo[2 * k] + I * Goo[2 * k + 1]) / a;",
     "cplx goo = (Goo[2 * k] + I * Goo[2 * k + 1]);"),
    ("determinant: sign of G_oo G_vv", "cplx dk = (1.0 + gov) * (1.0 + gvo) - goo * gvv;",
     "cplx dk = (1.0 + gov) * (1.0 + gvo) + goo * gvv;"),
    ("phase: principal branch per node", "phi[k] = phi[k + 1] + carg(r);",
     "phi[k] = carg(d[2 * k] + I * d[2 * k + 1]) + 0.0 * carg(r);"),
    ("quadrature: sin weight dropped", "s += fermi(beta, e, mu) * sin(thk) * phi[k];",
     "s += fermi(beta, e, mu) * phi[k];"),
    ("Fermi function sign", "double x = beta * (e - mu);", "double x = beta * (mu - e);"),
    ("Metropolis threshold", "int32_t own = (ds <= 0.0 || u < exp(-ds)) ? 1 : 0;",
     "int32_t own = (ds <= 0.0 || u < exp(ds)) ? 1 : 0;"),
    ("cone half-angle", "double ca = 1.0 - (1.0 - cos(p->cone)) * ua;",
     "double ca = 1.0 - (1.0 - cos(2.0 * p->cone)) * ua;"),
    ("random fraction count", "int64_t nr = (int64_t)floor(frac * (double)N);",
     "int64_t nr = (int64_t)ceil(frac * (double)N) + 1;"),
    ("magnetization: y component", "sy += sin(th[i]) * sin(ph[i]);", "sy += sin(th[i]) * cos(ph[i]);"),
    ("mixed vectors: o - iv", "const cplx cv[4] = {0.0, 1.0, 1.0, I};",
     "const cplx cv[4] = {0.0, 1.0, 1.0, -I};"),
    ("mixed formula: factor 1/2 dropped",
     "cplx gov = 0.5 * (gp - goo - gvv + I * (goo + gvv - gi));",
     "cplx gov = (gp - goo - gvv + I * (goo + gvv - gi));"),
]


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    d = tmp_path_factory.mktemp("mutants")
    yield d
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(workdir, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site not found: {old!r}"
    mutated = src.replace(old, new, 1)
    tag = "".join(c if c.isalnum() else "_" for c in name)
    csrc, lib = workdir / f"{tag}.c", workdir / f"lib{tag}.so"
    csrc.write_text(mutated)
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-I",
                           os.path.dirname(SRC), "-o", str(lib),
                           str(csrc), "-lm"])
    env = dict(os.environ, GFMC_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests",
                        "test_oracle_pins.py"), "-x", "-q", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"no pin failed for the planted mistake '{name}'"
