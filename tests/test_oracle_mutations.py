"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's source (a dropped term, a
wrong sign, coefficient, index, root or direction), builds it on the CPU, and
runs the oracle pin suite against that build: the suite must fail.  The real
oracle is untouched; the broken copies live in a temporary directory.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "rlb_oracle.cpp")
PINS = [os.path.join(ROOT, "tests", f) for f in
        ("test_oracle_pins.py", "test_oracle_riemann.py", "test_oracle_gradients.py",
         "test_oracle_transport.py", "test_oracle_eos.py", "test_oracle_positivity.py")]

MUTATIONS = {
    "drop_quadratic_term": ("6.0 * cu * cu / (cl2 * cl2)", "0.0 * cu * cu / (cl2 * cl2)"),
    "flip_u2_sign": ("6.0 * cu * cu / (cl2 * cl2) -\n                2.0 * u2 / cl2",
                     "6.0 * cu * cu / (cl2 * cl2) +\n                2.0 * u2 / cl2"),
    "rest_constant": ("(4.0 - (2.0 + cl2)", "(3.0 - (2.0 + cl2)"),
    "f_eq_coefficient": ("(1.0 + 3.0 * cu / cl2)", "(1.0 + 2.0 * cu / cl2)"),
    "diagonal_weight": ("return 1.0 / 36.0;", "return 1.0 / 18.0;"),
    "opposite_is_self": ("if (EV[p][0] == -EV[q][0] && EV[p][1] == -EV[q][1] && EV[p][2] == -EV[q][2]) return p;",
                         "if (p == q) return p;"),
    "push_instead_of_pull": ("L.resolve(a, c[a] - EV[q][a])", "L.resolve(a, c[a] + EV[q][a])"),
    "wrong_root": ("T W = (2.0 * E + sqrt(disc)) / 3.0;", "T W = (2.0 * E - sqrt(disc)) / 3.0;"),
    "relax_with_tau": ("og[q] = pg[q] - (1.0 / tau) * (pg[q] - geq[q]);",
                       "og[q] = pg[q] - (1.0 / (tau + 0.5)) * (pg[q] - geq[q]);"),
    "transposed_momentum_index": ("m0 += g[q] * (c_l * EV[q][0]);", "m0 += g[q] * (c_l * EV[q][1]);"),
    "outflow_wraps": ("if (bc[a][0] == BC_PERIODIC) return", "if (bc[a][0] != BC_INFLOW) return"),
    "gamma_sign": ("T gamma2 = 1.0 / (1.0 - u2);", "T gamma2 = 1.0 / (1.0 + u2);"),
    "transposed_jacobian": ("for (int q = 0; q < Q; ++q) mu += lam[q] * J[q][p];",
                            "for (int q = 0; q < Q; ++q) mu += lam[q] * J[p][q];"),
    "inflow_not_held": ("      if (bc[a][0] == BC_INFLOW && c[a] == 0) return true;",
                        "      if (bc[a][0] == BC_INFLOW && c[a] == 0 && false) return true;"),
    "eta_without_half_step": ("(tau * dt - dt / 2.0)", "(tau * dt)"),
    "entropy_log_sign": ("*s = 4.0 * n - n * log(lam);", "*s = 4.0 * n + n * log(lam);"),
    "n_eq_power": ("T n_eq = d_G * Tm * Tm * Tm / (pi * pi);", "T n_eq = d_G * Tm * Tm / (pi * pi);"),
    "temperature_coefficient": ("T Tm = eps / (3.0 * n);", "T Tm = eps / (4.0 * n);"),
    "tau_cell_by_instance": ("T tau = rx.tau_cell ? rx.tau_cell[i] : rx.tau[b];",
                             "T tau = rx.tau_cell ? rx.tau_cell[b] : rx.tau[b];"),
    "eta_s_rule_uses_n": ("T eta = eta_s * s;", "T eta = eta_s * n;"),
    "tau_cell_gradient_overwritten": ("if (dtau_cell) dtau_cell[i] += s;",
                                      "if (dtau_cell) dtau_cell[i] = s;"),
    "eos_pressure_term": ("(3.0 * P / ((P + eps) * gamma2 * cl2)",
                          "(2.0 * P / ((P + eps) * gamma2 * cl2)"),
    "eos_rest_coefficient": ("3.0 * P * (2.0 + cl2)", "3.0 * P * (1.0 + cl2)"),
    "eos_root_sign": ("T W = ((1.0 + kappa) * E + sqrt(disc)) / 2.0;",
                      "T W = ((1.0 + kappa) * E - sqrt(disc)) / 2.0;"),
    "positivity_mark_not_carried": ("if (trk && trk->mark[s.idx]) marked = true;",
                                    "if (trk && trk->mark[s.idx] && false) marked = true;"),
    "positivity_bound_coefficient": ("if (!(1.0 + 3.0 * cu / cl2 > 0.0)) return false;",
                                     "if (!(1.0 + 2.0 * cu / cl2 > 0.0)) return false;"),
    "update_cells_drops_kappa": ("collide<double>(pf, pg, tau, L.c_l, true, o, o + Q, L.kappa);",
                                 "collide<double>(pf, pg, tau, L.c_l, true, o, o + Q);"),
    "eos_energy_from_W": ("*eps = W / ((1.0 + kappa) * gamma2);",
                          "*eps = W / ((1.0 + kappa) * gamma2 * gamma2);"),
}


@pytest.fixture(scope="module")
def source():
    return open(SRC).read()


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, source, tmp_path):
    old, new = MUTATIONS[name]
    assert source.count(old) >= 1, f"mutation site for {name} not found"
    src = tmp_path / "mutant.cpp"
    src.write_text(source.replace(old, new, 1))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o",
                    str(lib), str(src)], check=True, capture_output=True)
    env = dict(os.environ, RLB_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"no pin caught the planted mistake '{name}':\n{r.stdout[-2000:]}"


def test_unmutated_copy_passes(source, tmp_path):
    """Control: the same build of the unmodified source passes the pin suite, so a
    failure above is the planted mistake's doing."""
    src = tmp_path / "copy.cpp"
    src.write_text(source)
    lib = tmp_path / "libcopy.so"
    subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o",
                    str(lib), str(src)], check=True, capture_output=True)
    env = dict(os.environ, RLB_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:]
