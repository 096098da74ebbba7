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

# planted mistakes in the open inlet/outlet planes, against their own pins
OPEN_MUTANTS = [
    ("open_mirror_to_periodic", "    if (outside(p, x, i, +1))\n        return node(p, x - EX[i]",
     "    if (0 && outside(p, x, i, +1))\n        return node(p, x - EX[i]"),
    ("open_neem_interior_density", "orc_equilibrium(rho_b, uf, eb);", "orc_equilibrium(rf[sig], uf, eb);"),
    ("open_held_wrong_directions", "if (EX[i] == dir_in)", "if (EX[i] == -dir_in)"),
    ("open_neem_velocity_component", "                        j[1] += EY[i] * fi;",
     "                        j[1] += EX[i] * fi;"),
]

# planted mistakes in the smooth non-wetting saturation (the adjoint's loss)
LOSS_MUTANTS = [
    ("loss_skips_rest_population", "for (int i = 0; i < Q; ++i) r[s] += f[((size_t)s * Q + i) * N + n];",
     "for (int i = 1; i < Q; ++i) r[s] += f[((size_t)s * Q + i) * N + n];"),
    ("loss_wrong_component", "acc += r[0] / (r[0] + r[1]);", "acc += r[1] / (r[0] + r[1]);"),
    ("loss_counts_solid", "if (solid[n] || !region[n]) continue;", "if (!region[n]) continue;"),
    ("loss_ignores_region", "if (solid[n] || !region[n]) continue;", "if (solid[n]) continue;"),
]

# planted mistakes in the diagnostics (masses, S_w, largest speed, non-finite count)
DIAG_MUTANTS = [
    ("diag_water_is_component_1", "if (r2 > r1) nw += 1.0;", "if (r1 > r2) nw += 1.0;"),
    ("diag_ties_count_as_water", "if (r2 > r1) nw += 1.0;", "if (r2 >= r1) nw += 1.0;"),
    ("diag_counts_solid", "        if (solid[n]) continue;\n        double r1 = rho[n], r2 = rho[N + n];\n        m1 += r1;",
     "        double r1 = rho[n], r2 = rho[N + n];\n        m1 += r1;"),
    ("diag_speed_misses_z", " + u[2 * N + n] * u[2 * N + n]);", ");"),
    ("diag_nonfinite_skips_rest", "            for (int i = 0; i < Q; ++i)\n                if (!isfinite",
     "            for (int i = 1; i < Q; ++i)\n                if (!isfinite"),
]

PIN_TESTS = [os.path.join(ROOT, "tests", "test_oracle_pins.py"),
             os.path.join(ROOT, "tests", "test_oracle_physics.py") + "::test_single_fluid_poiseuille"]


OPEN_PIN_TESTS = [os.path.join(ROOT, "tests", "test_oracle_open.py")]
LOSS_PIN_TESTS = [os.path.join(ROOT, "tests", "test_oracle_loss.py")]
DIAG_PIN_TESTS = [os.path.join(ROOT, "tests", "test_oracle_diagnostics.py")]


@pytest.mark.parametrize("name,orig,planted,pins",
                         [m + (PIN_TESTS,) for m in MUTANTS] + [m + (OPEN_PIN_TESTS,) for m in OPEN_MUTANTS]
                         + [m + (LOSS_PIN_TESTS,) for m in LOSS_MUTANTS]
                         + [m + (DIAG_PIN_TESTS,) for m in DIAG_MUTANTS],
                         ids=[m[0] for m in MUTANTS + OPEN_MUTANTS + LOSS_MUTANTS + DIAG_MUTANTS])
def test_planted_mistake_is_caught(name, orig, planted, pins, tmp_path):
    src = open(SRC).read()
    assert src.count(orig) == 1, name
    mut_src = tmp_path / "mut.c"
    mut_src.write_text(src.replace(orig, planted))
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", str(mut_src),
                    "-o", str(lib), "-lm"], check=True)
    env = dict(os.environ, MCLBM_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"]
                       + pins, cwd=ROOT, env=env, capture_output=True, text=True)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
