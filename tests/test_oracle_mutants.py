"""The oracle's pins must catch plausible mistakes: each mutant below plants one mistake in a
copy of the oracle source (a dropped term, a wrong sign or index, a transposed operand, an
off-by-one), builds it, and runs the pin suites against it; every mutant must fail them."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dogm_oracle.c")
PIN_SUITES = ["tests/test_oracle_rng.py", "tests/test_oracle_steps.py",
              "tests/test_oracle_recursion.py", "tests/test_oracle_bayes.py",
              "tests/test_oracle_exact_cycle.py"]

MUTANTS = {
    "predict_uses_vy_for_x": ("p->dt * vx[i] + p->sigma_pos * nz[0]",
                              "p->dt * vy[i] + p->sigma_pos * nz[0]"),
    "persistence_dropped": ("w[i] = p->p_s * w[i];", "w[i] = w[i];"),
    "cell_key_transposed": ("(uint32_t)floor(fy) * (uint32_t)p->nx + (uint32_t)floor(fx)",
                            "(uint32_t)floor(fx) * (uint32_t)p->ny + (uint32_t)floor(fy)"),
    "philox_weyl_constant": ("k1 += 0xBB67AE85u;", "k1 += 0xBB67AE86u;"),
    "box_muller_sin_cos_swapped": ("*n1 = radius * cos(two_pi * u2);\n    *n2 = radius * sin(two_pi * u2);",
                                   "*n1 = radius * sin(two_pi * u2);\n    *n2 = radius * cos(two_pi * u2);"),
    "dempster_dropped_term": ("(o1 * o2 + o1 * u2 + u1 * o2) / norm",
                              "(o1 * o2 + o1 * u2) / norm"),
    "free_mass_not_limited": ("pf_cand < 1.0 - po ? pf_cand : 1.0 - po", "pf_cand"),
    "birth_split_posterior_mass": ("rb = den > 0.0 ? o * a / den : 0.0;",
                                   "rb = den > 0.0 ? po * a / den : 0.0;"),
    "birth_everywhere": ("if (z_occ[c] > 0.0) {", "if (z_occ[c] >= 0.0) {"),
    "normaliser_missing_sum": ("double mua = s > 0.0 ? rho_p[c] / s : 0.0;",
                               "double mua = s > 0.0 ? rho_p[c] : 0.0;"),
    "assoc_weight_missing_pA": ("pa * rho_b[c] / (double)na", "rho_b[c] / (double)na"),
    "born_alloc_inclusive_scan": ("double o = floor((double)E * (double)nb / (double)S);",
                                  "double o = floor((double)(E + or_fixed40(rho_b[c])) * (double)nb / (double)S);"),
    "born_alloc_trailing_share_rounded": ("if (o > (double)nb || E >= S) o = (double)nb;",
                                          "if (o > (double)nb) o = (double)nb;"),
    "init_velocity_uses_process_noise": ("vx[i] = p->sigma_birth_vel * n0;",
                                         "vx[i] = p->sigma_vel * n0;"),
    "init_x_spans_ny": ("x[i] = or_uniform(b[0]) * (double)p->nx * p->cell_size;",
                        "x[i] = or_uniform(b[0]) * (double)p->ny * p->cell_size;"),
    "init_vy_repeats_vx_normal": ("vy[i] = p->sigma_birth_vel * n1;",
                                  "vy[i] = p->sigma_birth_vel * n0;"),
    "init_weight_uniform": ("        w[i] = 0.0;\n    }\n}", "        w[i] = 1.0 / (double)n;\n    }\n}"),
    "moments_mean_y_from_x": ("double mx = sx / r, my = sy / r;", "double mx = sx / r, my = sx / r;"),
    "variance_sign": ("var_x[c] = sxx / r - mx * mx;", "var_x[c] = sxx / r + mx * mx;"),
    "resample_off_by_one": ("while (i < N && F[i] <= t) ++i;", "while (i < N && F[i] < t) ++i;"),
    "resample_weight_wrong_count": ("return (double)W_fixed * 0x1p-40 / (double)nu;",
                                    "return (double)W_fixed * 0x1p-40 / (double)(nu + 1);"),
    "pignistic_half_dropped": ("pign[c] = o + 0.5 * (1.0 - o - f);", "pign[c] = o + (1.0 - o - f);"),
    "born_x_from_row": ("bx[s] = ((double)ix + u0) * p->cell_size;",
                        "bx[s] = ((double)iy + u0) * p->cell_size;"),
    "covariance_mean_x_twice": ("cov_xy[c] = sxy / r - mx * my;", "cov_xy[c] = sxy / r - mx * mx;"),
    # the particle PHD/MIB cell step (Sec. V)
    "phd_births_dropped": ("const double rb = p->p_b * (1.0 - rp);", "const double rb = 0.0;"),
    "phd_detection_tp_fp_swapped": ("f = p_tp[c] / (p_fp[c] * (1.0 - r) + p_tp[c] * r);",
                                    "f = p_fp[c] / (p_tp[c] * (1.0 - r) + p_fp[c] * r);"),
    "phd_miss_wrong_complement": ("((1.0 - p_tp[c]) * r + (1.0 - p_fp[c]) * (1.0 - r))",
                                  "((1.0 - p_tp[c]) * r + (1.0 - p_fp[c]) * r)"),
    "phd_no_truncation": ("const double rp = s < 1.0 ? s : 1.0;", "const double rp = s;"),
    "phd_rho_p_unscaled": ("rho_p[c] = f * rp;", "rho_p[c] = rp;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                           str(mpath), "-o", str(lib), "-lm"])
    env = dict(os.environ, DOGM_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PIN_SUITES], cwd=ROOT, env=env, capture_output=True, text=True)
    assert r.returncode == 1, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
