"""The oracle's pins have teeth: plant one plausible mistake at a time in a copy
of the oracle source (CPU only), build it, and check that the pin suite fails.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mclbm_oracle.c")

# (name, original text, planted mistake)
MUTANTS = [
    ("wrong_diagonal_weight", "1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,\n",
     "1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,\n"),
    ("transposed_velocity_entry", "static const int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};",
     "static const int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, 1, -1, -1};"),
    ("source_sign", "((e[a] - u[a]) / CS2", "((e[a] + u[a]) / CS2"),
    ("dropped_quadratic_term", " + (eu * eu) / (2.0 * CS2 * CS2)", ""),
    ("bounce_back_same_direction", "v = f_in[((size_t)s * Q + opp[i]) * N + n];",
     "v = f_in[((size_t)s * Q + i) * N + n];"),
    ("chi_swapped", "double chi[NC] = {1.0 + xi[n], 1.0 - xi[n]};",
     "double chi[NC] = {1.0 - xi[n], 1.0 + xi[n]};"),
    ("force_index_transposed", "sum[2] += W[i] * ps * EZ[i];", "sum[2] += W[i] * ps * EY[i];"),
    ("own_component_in_force", "int sb = 1 - s; /* the other component */", "int sb = s;"),
    ("viscosity_plus_sign", "return CS2 * (tau - 0.5);", "return CS2 * (tau + 0.5);"),
    ("body_force_dropped", "-p->G * r * sum[a] + r * p->g[s][a]", "-p->G * r * sum[a]"),
    ("half_force_weight", "mom[a] += 0.5 * F", "mom[a] += 1.0 * F"),
    ("ivsd_includes_solid", "double fluid = solid[m] ? 0.0 : 1.0; /* 1 - phi */",
     "double fluid = 1.0;"),
]

PIN_TESTS = [os.path.join(ROOT, "tests", "test_oracle_pins.py"),
             os.path.join(ROOT, "tests", "test_oracle_physics.py") + "::test_single_fluid_poiseuille"]


@pytest.mark.parametrize("name,orig,planted", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(name, orig, planted, tmp_path):
    src = open(SRC).read()
    assert src.count(orig) == 1, name
    mut_src = tmp_path / "mut.c"
    mut_src.write_text(src.replace(orig, planted))
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", str(mut_src),
                    "-o", str(lib), "-lm"], check=True)
    env = dict(os.environ, MCLBM_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"]
                       + PIN_TESTS, cwd=ROOT, env=env, capture_output=True, text=True)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
