"""The oracle's pins are sensitive: each plausible mistake planted in a copy of
oracle.c (a dropped term, a wrong sign, a wrong index or branch, a swapped
rate) makes at least one pin of the CPU suite fail.

The mutated copies are compiled into a temporary directory and loaded through
LBM_ORACLE_LIB in a child pytest run; the committed oracle is never changed.
"""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
PINS = [os.path.join(ROOT, "tests", "test_oracle_equilibria.py"),
        os.path.join(ROOT, "tests", "test_oracle_physics.py"),
        os.path.join(ROOT, "tests", "test_oracle_caloric.py")]

MUTANTS = [
    ("psi_minus_sign", "return 0.5 * (-xi + P);", "return 0.5 * (xi + P);"),
    ("anomaly_temperature_factor", "rho * u * (1.0 - 3.0 * T)", "rho * u * (1.0 - T)"),
    ("extended_P_drops_rho", "(2.0 - omega) / (2.0 * rho * omega) * d[a]", "(2.0 - omega) / (2.0 * omega) * d[a]"),
    ("extended_P_no_correction", "(2.0 - omega) / (2.0 * rho * omega) * d[a]", "0.0 * d[a]"),
    ("upwind_branch_reversed", "if (u[n] > 0.0) {", "if (u[n] < 0.0) {"),
    ("dq_anomaly_sign", "double divQ = (a == b) ? 0.5 * d[a] : 0.0;", "double divQ = (a == b) ? -0.5 * d[a] : 0.0;"),
    ("dq_transposed_u", "s += u[b] * (P[b * D + a] - Peq + divQ);", "s += u[a] * (P[b * D + a] - Peq + divQ);"),
    ("g_relaxes_with_omega", "g_out[i] = gh[i] + m->omega1 * (geq[i] - gh[i])",
     "g_out[i] = gh[i] + m->omega * (geq[i] - gh[i])"),
    ("quasi_eq_wrong_directions", "g[i] = (c2 == 1) ? geq[i] + 0.5 * cdq : geq[i];",
     "g[i] = (c2 == 2) ? geq[i] + 0.5 * cdq : geq[i];"),
    ("quasi_eq_sign", "(m->omega - m->omega1) * (geq[i] - gst[i])", "(m->omega - m->omega1) * (gst[i] - geq[i])"),
    ("omega1_formula", "2.0 * Pr * omega / (2.0 - omega + Pr * omega)", "2.0 * Pr * omega / (2.0 + omega - Pr * omega)"),
    ("operator_drops_power", "r.c[k - 1] += T * (double)k * A->c[k];", "r.c[k - 1] += T * A->c[k];"),
    ("temperature_kinetic_term", "m->T = orc_temperature(cv, E - 0.5 * u2);", "m->T = orc_temperature(cv, E - u2);"),
    ("stream_wrong_direction", "long sh[3] = {-c[0], -c[1], -c[2]};", "long sh[3] = {c[0], c[1], c[2]};"),
    ("clamp_off_by_one", "if (r > n - 1) r = n - 1;", "if (r > n - 1) r = n - 2;"),
    ("power_law_inverted", "pow(T / p->T_ref, p->visc_exp)", "pow(p->T_ref / T, p->visc_exp)"),
    ("central_half_dropped", "out[n] = 0.5 * (Qt[np] - Qt[nm]);", "out[n] = (Qt[np] - Qt[nm]);"),
    ("viscosity_uses_pressure_wrong", "return 1.0 / (mu / (rho * T) + 0.5);", "return 1.0 / (mu / rho + 0.5);"),
    ("internal_energy_half_dropped", "cv[1] * T * T / 2.0", "cv[1] * T * T"),
    ("newton_step_sign", "    T -= dT;", "    T += dT;"),
    ("geq_ignores_caloric_law", "double s = U;", "double s = 2.5 * T;"),
    ("sound_speed_gamma_inverted", "gam = (cvT + 1.0) / cvT;", "gam = cvT / (cvT + 1.0);"),
]


def _run_mutant(name, old, new, tmp):
    src = open(SRC).read()
    assert src.count(old) == 1, f"{name}: target not unique in oracle.c"
    path = os.path.join(tmp, f"{name}.c")
    with open(path, "w") as fh:
        fh.write(src.replace(old, new))
    lib = os.path.join(tmp, f"lib_{name}.so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-I",
                           os.path.join(ROOT, "oracle"), "-o", lib, path, "-lm"])
    env = dict(os.environ, LBM_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode


def test_every_planted_mistake_is_caught():
    with tempfile.TemporaryDirectory() as tmp:
        with cf.ThreadPoolExecutor(max_workers=4) as ex:
            results = list(ex.map(lambda m: _run_mutant(*m, tmp), MUTANTS))
    survivors = [name for name, rc in results if rc == 0]
    assert not survivors, f"pins did not catch: {survivors}"
