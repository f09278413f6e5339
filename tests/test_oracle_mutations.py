"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle (a dropped term, a wrong
sign, a wrong power, a transposed operand, a wrong tableau entry, a wrong
step-control constant or norm, a wrong unit factor), builds it on the CPU, and
runs the pin suite against it: mistakes in nh_oracle.c through NH_ORACLE_LIB
(a mutated build of the C file), mistakes in oracle.py through NH_ORACLE_ROOT
(a directory holding a mutated copy of the oracle package, imported first).
The suite must fail for every mutant.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "nh_oracle.c")
PY_SRC = os.path.join(ROOT, "oracle", "oracle.py")

MUTANTS = {
    "force_sign": ("dY[2] = -g * x;", "dY[2] = g * x;"),
    "force_transposed": ("dY[3] = -g * y;", "dY[3] = -g * x;"),
    "drift_power": ("A = opz * opz / H;", "A = opz / H;"),
    "kick_factor": ("B = nho_kappa(m, z) * nho_G() * opz / H;", "B = nho_kappa(m, z) * nho_G() / H;"),
    "no_compensation": ("if (r < rv) return Mz * (nho_nfw_I(r / s) / nho_nfw_I(c) - comp);",
                        "if (r < rv) return Mz * (nho_nfw_I(r / s) / nho_nfw_I(c));"),
    "shell_sign": ("return Mz * (1.0 - comp);", "return Mz * (1.0 + comp);"),
    "nfw_I_term": ("return log1p(q) - q / (1.0 + q);", "return log1p(q) - q;"),
    "series_sign": ("sum += (k % 2 == 0) ? term : -term;", "sum += term;"),
    "hubble_power": ("sqrt(m->Omega_m * opz * opz * opz + m->Omega_L)", "sqrt(m->Omega_m * opz * opz + m->Omega_L)"),
    "lagrangian_radius": ("double fac = 2.0 * nho_G() / (m->Omega_m * H0k * H0k);",
                          "double fac = 3.0 * nho_G() / (m->Omega_m * H0k * H0k);"),
    "truncation_image": ("*rv = (*R / c200) * ((1.0 + z) / (1.0 + m->z_obs));", "*rv = (*R / c200);"),
    "rk4_weight": ("(k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i])", "(k1[i] + 2.0 * k2[i] + k3[i] + 2.0 * k4[i])"),
    "rk4_stage_time": ("nho_rhs(m, u1, T, k3);", "nho_rhs(m, u0, T, k3);"),
    "dp_tableau": ("{44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0},", "{44.0 / 45.0, -56.0 / 15.0, 32.0 / 8.0, 0, 0, 0},"),
    "dp_weight": ("static const double DP_B[7] = {35.0 / 384.0,", "static const double DP_B[7] = {36.0 / 384.0,"),
    "dp_error_weight": ("-92097.0 / 339200.0, 187.0 / 2100.0, 1.0 / 40.0};", "-92097.0 / 339200.0, 187.0 / 2100.0, 1.0 / 30.0};"),
    "mass_xi": ("double xi = (m->z_form - z) / (m->z_form - m->z_obs);",
                "double xi = (m->z_form - z) / (m->z_form + 1.0 - m->z_obs);"),
    "observed_truncation": ("*rv = (*R / c200) * ((1.0 + z) / (1.0 + m->z_obs));", "*rv = (*R / c200) * (1.0 + z);"),
    "observed_radius": ("*R = cbrt(fac * nho_mass(m, m->z_obs));", "*R = cbrt(fac * nho_mass(m, 0.0));"),
    "conc_power": ("return m->c0 * pow(1.0 + z, -m->conc_gamma);", "return m->c0 * pow(1.0 + z, m->conc_gamma);"),
    "sampled_horner": ("return ((c[0] * t + c[1]) * t + c[2]) * t + c[3];",
                       "return ((c[0] * t + c[2]) * t + c[1]) * t + c[3];"),
    "sampled_piece_origin": ("double t = u - (m->hist_u_min + (double)i * du);",
                             "double t = u - (m->hist_u_min + (double)(i + 1) * du);"),
    "sampled_time_sign": ("double u = -log1p(z);\n    double du", "double u = log1p(z);\n    double du"),
    "sampled_spacing": ("double du = (0.0 - m->hist_u_min) / (double)(m->hist_n - 1);",
                        "double du = (0.0 - m->hist_u_min) / (double)m->hist_n;"),
    # step control (Hairer, Norsett & Wanner, Sec. II.4, as read for the paper's unstated integrator)
    "dp_no_cap_after_rejection": ("            if (rejected_prev && fac > 1.0) fac = 1.0;\n", ""),
    "dp_max_norm": ("for (int i = 0; i < 4; ++i) { double e = E[i] / sc[i]; sum += e * e; }",
                    "for (int i = 0; i < 4; ++i) { double e = E[i] / sc[i]; if (4.0 * e * e > sum) sum = 4.0 * e * e; }"),
    "dp_fmax_10": ("const double fmax = it->fmax > 0.0 ? it->fmax : 5.0;",
                   "const double fmax = it->fmax > 0.0 ? it->fmax : 10.0;"),
    "dp_safety_accept": ("double fac = (err == 0.0) ? fmax : 0.9 * pow(err, -0.2);",
                         "double fac = (err == 0.0) ? fmax : 0.8 * pow(err, -0.2);"),
    "dp_position_scale_max_component": (
        "sc[0] = sc[1] = it->atol_x + it->rtol * (rx0 > rx1 ? rx0 : rx1);",
        "sc[0] = sc[1] = it->atol_x + it->rtol * (fabs(Y[0]) > fabs(Y5[0]) ? fabs(Y[0]) : fabs(Y5[0]));"),
}

# Mistakes in the Python half of the oracle (initial conditions, quadrature).
PY_MUTANTS = {
    "velocity_scale": ("    return K_B_EV_PER_K * T_K * C_KM_S / m_eV",
                       "    return 1.5 * K_B_EV_PER_K * T_K * C_KM_S / m_eV"),
    "velocity_temperature": ("    return K_B_EV_PER_K * T_K * C_KM_S / m_eV",
                             "    return K_B_EV_PER_K * C_KM_S / m_eV"),
    "trapezoid_end_weight": ("        d[0] = 0.5 * (ly[1] - ly[0])", "        d[0] = (ly[1] - ly[0])"),
}


def _run_pins(env):
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                          env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "mut.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                    "-o", str(so), str(mut), "-lm"], check=True)
    r = _run_pins(dict(os.environ, NH_ORACLE_LIB=str(so)))
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_pins_catch_python_mutant(name, tmp_path):
    old, new = PY_MUTANTS[name]
    src = open(PY_SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    (pkg / "oracle.py").write_text(src.replace(old, new))
    shutil.copy(SRC, pkg / "nh_oracle.c")
    env = dict(os.environ, NH_ORACLE_ROOT=str(tmp_path))
    env.pop("NH_ORACLE_LIB", None)
    r = _run_pins(env)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"


def test_unmutated_copies_pass(tmp_path):
    """Control: both routes, given the oracle unchanged, pass the pins (so a
    mutant fails because of its mistake, not because of the route)."""
    so = tmp_path / "same.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                    "-o", str(so), SRC, "-lm"], check=True)
    r = _run_pins(dict(os.environ, NH_ORACLE_LIB=str(so)))
    assert r.returncode == 0, r.stdout[-2000:]
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    shutil.copy(PY_SRC, pkg / "oracle.py")
    shutil.copy(SRC, pkg / "nh_oracle.c")
    env = dict(os.environ, NH_ORACLE_ROOT=str(tmp_path))
    env.pop("NH_ORACLE_LIB", None)
    r = _run_pins(env)
    assert r.returncode == 0, r.stdout[-2000:]
