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
PINS = [os.path.join(ROOT, "tests", "test_oracle_diagnostics.py"),
        os.path.join(ROOT, "tests", "test_oracle_sampled.py"),
        os.path.join(ROOT, "tests", "test_oracle_equilibria.py"),
        os.path.join(ROOT, "tests", "test_oracle_physics.py"),
        os.path.join(ROOT, "tests", "test_oracle_caloric.py")]

MUTANTS = [
    ("psi_minus_sign", "return 0.5 * (-xi + P);", "return 0.5 * (xi + P);"),
    ("anomaly_temperature_factor", "rho * u * (1.0 - 3.0 * T)", "rho * u * (1.0 - T)"),
    ("extended_P_drops_rho", "(2.0 - omega) / (2.0 * rho * omega) * d[a]", "(2.0 - omega) / (2.0 * omega) * d[a]"),
    ("extended_P_no_correction", "(2.0 - omega) / (2.0 * rho * omega) * d[a]", "0.0 * d[a]"),
    ("upwind_branch_reversed", "int backward = u[n] > 0.0;", "int backward = u[n] < 0.0;"),
    ("upwind_band_ignored", "if (s->band > 0.0 && fabs(u[n]) <= s->band) backward = !backward;",
     "if (s->band < 0.0 && fabs(u[n]) <= s->band) backward = !backward;"),
    ("upwind_band_flips_zero", "if (s->band > 0.0 && fabs(u[n]) <= s->band) backward = !backward;",
     "if (fabs(u[n]) <= s->band) backward = !backward;"),
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
    # diagnostics (Eqs. (3)-(5), Sec. III.D statistics)
    ("kinetic_energy_doubled", "c[(size_t)ORC_D_KINETIC * N] = 0.5 * rho[n] * uu;",
     "c[(size_t)ORC_D_KINETIC * N] = rho[n] * uu;"),
    ("diagnostic_central_half_dropped",
     "return 0.5 * (F[neighbour(&s->p, n, axis, +1)] - F[neighbour(&s->p, n, axis, -1)]);",
     "return (F[neighbour(&s->p, n, axis, +1)] - F[neighbour(&s->p, n, axis, -1)]);"),
    ("curl_z_sign", "gz = central(s, u + (size_t)N, n, 0) - central(s, u, n, 1);",
     "gz = central(s, u + (size_t)N, n, 0) + central(s, u, n, 1);"),
    ("curl_x_sign", "gx = central(s, u + 2 * (size_t)N, n, 1) - central(s, u + (size_t)N, n, 2);",
     "gx = central(s, u + 2 * (size_t)N, n, 1) + central(s, u + (size_t)N, n, 2);"),
    ("curl_y_wrong_axis", "gy = central(s, u, n, 2) - central(s, u + 2 * (size_t)N, n, 0);",
     "gy = central(s, u, n, 1) - central(s, u + 2 * (size_t)N, n, 0);"),
    ("dilatation_last_axis_only", "div += du[a];", "div = du[a];"),
    ("dissipation_constant_mu", "c[(size_t)ORC_D_DISS * N] = viscosity(p, T[n]) * vort2;",
     "c[(size_t)ORC_D_DISS * N] = p->mu0 * vort2;"),
    ("rho2_not_squared", "c[(size_t)ORC_D_RHO2 * N] = rho[n] * rho[n];", "c[(size_t)ORC_D_RHO2 * N] = rho[n];"),
    ("u_axis_slot_index", "c[(size_t)ORC_D_UY2 * N] = uy * uy;", "c[(size_t)ORC_D_UY2 * N] = ux * ux;"),
    ("du_axis_slot_index", "c[(size_t)ORC_D_DUY2 * N] = du[1] * du[1];", "c[(size_t)ORC_D_DUY2 * N] = du[0] * du[0];"),
    ("nonpositive_ignores_rho", "(rho[n] <= 0.0 || T[n] <= 0.0)", "(T[n] <= 0.0)"),
    # sampled step, upwind-side override, FP32 storage model
    ("override_sides_swapped", "return side == 0 ? Qt[n] - Qt[nm] : Qt[np] - Qt[n];",
     "return side == 1 ? Qt[n] - Qt[nm] : Qt[np] - Qt[n];"),
    ("sampled_step_list_index", "pass2_node(&tmp, node, d, f_out + k, count, g_out + k, count);",
     "pass2_node(&tmp, k % tmp.N, d, f_out + k, count, g_out + k, count);"),
    ("sampled_step_derivative_axis", "d[a] = tmp.dd[(size_t)a * tmp.N + node];",
     "d[a] = tmp.dd[(size_t)(D - 1 - a) * tmp.N + node];"),
    ("storage_not_rounded", "*f = s->fref[i] + (double)(float)(*f - s->fref[i]);",
     "*f = s->fref[i] + (*f - s->fref[i]);"),
    ("storage_not_rounded_at_init", "  round_storage(s);\n  s->step = 0;", "  s->step = 0;"),
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
