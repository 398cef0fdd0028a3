"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of ``oracle/oracle.c`` (on the CPU,
in a temporary directory), builds it, and runs the pin suite against that
build.  The suite must fail for every planted mistake.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, original text, planted mistake)
MUTANTS = [
    ("arithmetic_mean_face", "kf = 2.0 * kp * kn / (kp + kn);", "kf = 0.5 * (kp + kn);"),
    ("geometric_mean_face", "kf = 2.0 * kp * kn / (kp + kn);", "kf = sqrt(kp * kn);"),
    ("dirichlet_half_cell", "const double D = p->dt * kp / (p->h * p->h);",
     "const double D = 2.0 * p->dt * kp / (p->h * p->h);"),
    ("dirichlet_neighbour_kappa_missing", "const double D = p->dt * kp / (p->h * p->h);",
     "const double D = p->dt * p->alpha / (p->h * p->h);"),
    ("conductance_over_h", "const double D = p->dt * kf / (p->h * p->h);",
     "const double D = p->dt * kf / p->h;"),
    ("upwind_reversed", "off[f] = -(D + fmax(-F, 0.0));", "off[f] = -(D + fmax(F, 0.0));"),
    ("upwind_central", "off[f] = -(D + fmax(-F, 0.0));", "off[f] = -(D - 0.5 * F);"),
    ("outflow_abs", "      diag += D + fmax(F, 0.0);\n      off[f]",
     "      diag += D + fabs(F);\n      off[f]"),
    ("flux_number_h2", "const double F = p->dt * (p->u[axis] * normal) / p->h;",
     "const double F = p->dt * (p->u[axis] * normal) / (p->h * p->h);"),
    ("bterm_no_inflow", "bterm += (D + fmax(-F, 0.0)) * p->bc_value[f];",
     "bterm += D * p->bc_value[f];"),
    ("dirichlet_outflow_dropped",
     "      const double D = p->dt * kp / (p->h * p->h);\n      diag += D + fmax(F, 0.0);",
     "      const double D = p->dt * kp / (p->h * p->h);\n      diag += D;"),
    ("zeroflux_as_dirichlet", "} else if (p->bc_kind[f] == ORC_DIRICHLET) {", "} else {"),
    ("rhs_sign", "b[c] = Tn[c] + bterm;", "b[c] = Tn[c] - bterm;"),
    ("neighbour_coefficient_swap",
     "if (j > 0)      acc += off[2] * x[cell_index(p, i, j - 1, k)];",
     "if (j > 0)      acc += off[3] * x[cell_index(p, i, j - 1, k)];"),
    ("neighbour_index_swap",
     "if (k < nz - 1) acc += off[5] * x[cell_index(p, i, j, k + 1)];",
     "if (k < nz - 1) acc += off[5] * x[cell_index(p, i, j + 1 < ny ? j + 1 : j, k)];"),
    ("beta_missing_alpha_over_omega", "const double beta = (rho / rho_prev) * (alpha / omega);",
     "const double beta = (rho / rho_prev);"),
    ("p_update_sign", "pv[c] = r[c] + beta * (pv[c] - omega * v[c]);",
     "pv[c] = r[c] + beta * (pv[c] + omega * v[c]);"),
    ("alpha_inverted", "alpha = rho / sigma;", "alpha = sigma / rho;"),
    ("omega_inverted", "omega = ts / tt;", "omega = tt / ts;"),
    ("x_update_drops_s", "x[c] = x[c] + alpha * pv[c] + omega * s[c];",
     "x[c] = x[c] + alpha * pv[c];"),
    ("r_update_sign", "r[c] = s[c] - omega * t[c];", "r[c] = s[c] + omega * t[c];"),
    ("s_update_sign", "s[c] = r[c] - alpha * v[c];", "s[c] = r[c] + alpha * v[c];"),
    ("absolute_stop_test", "if (rnorm <= tol * bn) { status = ORC_OK; goto done; }\n    if (omega",
     "if (rnorm <= tol) { status = ORC_OK; goto done; }\n    if (omega"),
    ("cg_beta_inverted", "const double beta = rr_new / rr;", "const double beta = rr / rr_new;"),
    ("cg_step_sign", "x[c] += a * d[c]; r[c] -= a * q[c];", "x[c] -= a * d[c]; r[c] -= a * q[c];"),
    ("cg1_step_ignores_beta", "const double denom = delta - beta * gamma_new / alpha;",
     "const double denom = delta;"),
    ("cg1_s_recurrence_dropped", "pv[c] = r[c] + beta * pv[c]; s[c] = w[c] + beta * s[c];",
     "pv[c] = r[c] + beta * pv[c]; s[c] = w[c];"),
    ("bicgstab2_beta_uses_exact_rho", "const double rho_pred = rs - omega * rt;",
     "const double rho_pred = rs + omega * rt;"),
    ("bicgstab2_x_update_order", "x[c] = x[c] + alpha * pv[c] + omega * sc;",
     "x[c] = x[c] + alpha * pv[c] + omega * r[c];"),
    ("bicgstab2_r_update_sign", "r[c] = sc - omega * t[c];", "r[c] = sc + omega * t[c];"),
    ("bicgstab2_p_update", "pv[c] = r[c] + beta * (pv[c] - omega * v[c]);\n      }",
     "pv[c] = r[c] + beta * pv[c];\n      }"),
    ("jacobi_multiplies", "y[cell_index(p, i, j, k)] /= diag;",
     "y[cell_index(p, i, j, k)] *= diag;"),
    ("jacobi_rhs_unscaled", "out[c] = b[c] / diag;", "out[c] = b[c];"),
    ("explicit_flux_sign", "T[c] = Tn[c] - flux + bterm;", "T[c] = Tn[c] + flux + bterm;"),
    ("explicit_keeps_identity", "double flux = (diag - 1.0) * Tn[c];",
     "double flux = diag * Tn[c];"),
    ("bicgstab2_shadow_ignored", "if (hashed_shadow) orc_shadow(n, rh);\n  else memcpy(rh, r, bytes);",
     "memcpy(rh, r, bytes);"),
    ("dot_drops_last_plane", "for (int k = 0; k < nz; ++k) total += part[k];",
     "for (int k = 0; k + 1 < nz; ++k) total += part[k];"),
    ("true_relres_zero", "return bn > 0.0 ? rn / bn : rn;", "return 0.0;"),
    ("true_relres_squared", "return bn > 0.0 ? rn / bn : rn;",
     "return bn > 0.0 ? (rn / bn) * (rn / bn) : rn;"),
    ("true_relres_absolute", "return bn > 0.0 ? rn / bn : rn;", "return rn;"),
    ("true_relres_residual_sign", "for (long c = 0; c < n; ++c) r[c] = b[c] - r[c];\n}\n\n/*\n * The operator",
     "for (long c = 0; c < n; ++c) r[c] = b[c] + r[c];\n}\n\n/*\n * The operator"),
    ("restart_breaks_down",
     "  do_restart:\n    if (++restarts > ORC_MAX_RESTARTS) { status = ORC_BREAKDOWN; goto done; }\n"
     "    goto restart;\n  }\n  status = ORC_NOCONV;",
     "  do_restart:\n    if (++restarts > 0) { status = ORC_BREAKDOWN; goto done; }\n"
     "    goto restart;\n  }\n  status = ORC_NOCONV;"),
    ("restart_keeps_old_shadow", "  memcpy(rh, r, bytes);\n  memset(pv, 0, bytes);",
     "  if (restarts == 0) memcpy(rh, r, bytes);\n  memset(pv, 0, bytes);"),
    ("restart_keeps_direction", "  memset(pv, 0, bytes);\n  memset(v, 0, bytes);",
     "  if (restarts == 0) { memset(pv, 0, bytes); memset(v, 0, bytes); }"),
    ("restart_counts_cut_iteration", "    --it;                                /* ended before its update of x */\n",
     ""),
    ("bicgstab2_restart_breaks_down",
     "    if (++restarts > ORC_MAX_RESTARTS) { status = ORC_BREAKDOWN; goto done; }\n"
     "    goto restart;\n  }\n\ndone:",
     "    if (++restarts > 0) { status = ORC_BREAKDOWN; goto done; }\n"
     "    goto restart;\n  }\n\ndone:"),
    ("bicgstab2_restart_keeps_old_shadow",
     "if (hashed_shadow) orc_shadow(n, rh);\n  else memcpy(rh, r, bytes);",
     "if (hashed_shadow) orc_shadow(n, rh);\n  else if (restarts == 0) memcpy(rh, r, bytes);"),
]


@pytest.mark.parametrize("name,orig,bad", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, orig, bad):
    src = open(SRC).read()
    assert src.count(orig) >= 1, f"mutation anchor for {name} not found"
    mutated = src.replace(orig, bad, 1)
    csrc = tmp_path / "oracle_mutant.c"
    csrc.write_text(mutated)
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", str(lib),
                    str(csrc), "-lm"], check=True)
    env = dict(os.environ, ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode != 0, f"pins did not catch mutant {name}:\n{res.stdout[-2000:]}"
