"""The oracle's pins catch plausible mistakes.

Each case copies the oracle source with one planted mistake (a flipped sign,
a dropped factor, a transposed operand, a wrong tie rule ...), builds it on
the CPU and runs the pin suite against it through TRD_ORACLE_LIB; the suite
must fail.  The real oracle passes the same suite in the other tests.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "trd_oracle.c")

MUTANTS = {
    "jacobian_dz_dc_sign": ("J[1][4] = k * t * arc * arc", "J[1][4] = -k * t * arc * arc"),
    "jacobian_dy_ds_f": ("J[0][2] = arc * sinc(delta) / (f1 * f2);", "J[0][2] = arc * sinc(delta) / (f1 * f1);"),
    "scattering_drops_f2": ("C[2][2] += th2 * f * f * tt;", "C[2][2] += th2 * tt;"),
    "transport_transposed": ("for (int k = 0; k < 5; k++) a += T[i][k] * J[j][k];",
                             "for (int k = 0; k < 5; k++) a += T[i][k] * J[k][j];"),
    "tilt_sign": ("double ry = yj - (ye + r->tau * (ze - zj));", "double ry = yj - (ye - r->tau * (ze - zj));"),
    "curvature_sign": ("double k = -KAPPA * g->bz;            /* d curvature / d (q/pT) */",
                       "double k = KAPPA * g->bz;"),
    "field_z_term_dropped": ("+ g->field_bz * z * z / (FIELD_ZREF * FIELD_ZREF));", ");"),
    "field_radius_local_x_only": ("const double r2 = x * x + y * y;", "const double r2 = x * x;"),
    "rk_weights": ("hs / 6.0 * (k1[j] + 2.0 * k2[j] + 2.0 * k3[j] + k4[j])",
                   "hs / 6.0 * (k1[j] + 2.0 * k2[j] + 2.0 * k2[j] + k4[j])"),
    "rotation_ds_dy_sign": ("J[2][0] = -cu * sa;", "J[2][0] = cu * sa;"),
    "dy_gate_slope_power": ("C[2][2] / (f3 * f3));", "C[2][2] / (f3));"),
    "chi2_cross_term": ("2.0 * r->Si[0][1] * ry * rz", "r->Si[0][1] * ry * rz"),
    "tie_to_higher_index": ("(c2 == bchi && j < best_orig)", "(c2 == bchi && j > best_orig)"),
    "bin_rounding": ("double u = floor((v - lo) * (1.0 / w));", "double u = floor((v - lo) * (1.0 / w) + 0.5);"),
    "joseph_drops_kvk": ("for (int a = 0; a < 2; a++)\n                for (int b = 0; b < 2; b++) v += K[i][a] * V[a][b] * K[j][b];", ""),
    "no_scattering": ("            add_ms(p, C, g);\n            if (!eloss(p, C, g, 1,", "            if (!eloss(p, C, g, 1,"),
    "beam_first_parent_state": ("*d = H[c->parent];", "*d = H[0];"),
    "beam_cost_not_carried": ("d->cost = c->cost;", ""),
    "beam_sum_holds_cost": ("d->chi2sum += c->chi2;", "d->chi2sum += c->cost;"),
    "refit_no_scattering": ("                add_ms(p, C, g);\n                eloss(p, C, g, -1, NULL);",
                            "                eloss(p, C, g, -1, NULL);"),
    "refit_chi2_cross_sign": ("(Szz * ry * ry - 2.0 * Syz * ry * rz + Syy * rz * rz) / det2",
                              "(Szz * ry * ry + 2.0 * Syz * ry * rz + Syy * rz * rz) / det2"),
    "refit_tilt_sign": ("const double ry = ky[j] - (p[0] + tau * (p[1] - kz[j]));",
                        "const double ry = ky[j] - (p[0] - tau * (p[1] - kz[j]));"),
    "residual_stt_drops_z": ("S[3] += ty * ty + tz * tz;", "S[3] += ty * ty;"),
    "residual_voxel_y_sign": ("double fy = (y / x / tan10 + 1.0) * 0.5 * t->ny;",
                              "double fy = (-y / x / tan10 + 1.0) * 0.5 * t->ny;"),
    "residual_solve_sign": ("const double b = -S[6] + (st * S[4] + sz * S[5]) / nn;",
                            "const double b = S[6] - (st * S[4] + sz * S[5]) / nn;"),
    "eloss_direction": ("double E2 = dir > 0 ? E - dE : E + dE;", "double E2 = dir > 0 ? E + dE : E - dE;"),
    "eloss_no_path_factor": ("* g->eloss_xrho * sqrt(tt) / f;", "* g->eloss_xrho;"),
    "eloss_jacobian_square": ("double j = k * k * k * E2 / E;", "double j = k * k * E2 / E;"),
    "bethe_drops_beta2": ("/ (g->eloss_i * g->eloss_i)) - b2);", "/ (g->eloss_i * g->eloss_i)));"),
    "refit_no_eloss": ("                eloss(p, C, g, -1, NULL);\n", ""),
    "absent_penalty_ignored": ("if (a0) pen = 0.0;", ""),
    "absent_not_dropped": ("!isfinite(dy) || g->absent[det])", "!isfinite(dy))"),
    "resolution_curvature_linear": ("a[1] * s + a[2] * s * s; }", "a[1] * s + a[2] * s; }"),
    "resolution_slope_sign": ("return a[0] + a[1] * s + a[2]", "return a[0] - a[1] * s + a[2]"),
    "lorentz_offset_sign": ("r.dytrk = g->drift_len * (r.tphi - g->tan_psi);",
                            "r.dytrk = g->drift_len * (r.tphi + g->tan_psi);"),
    "update_width_at_the_minimum": ("double syu = poly2(g->sigma_y, p[2]);", "double syu = g->sigma_y[0];"),
    "flag_margin_wider": ("return fabs(a - lim) <= rel * fabs(lim) + abs_;",
                          "return fabs(a - lim) <= 4.0 * rel * fabs(lim) + abs_;"),
    "flag_p2_any_loser": ("if (best < 0 || c2 <= bchi + g->m_rel * bchi + g->m_chi2 + chi2_err(&r, bchi) + chi2_err(&r, c2))",
                          "if (1)"),
    "flag_p2_two_gates": ("if (!fail || popcount4(fail) != 1 || !(fail & nm)) continue;",
                          "if (!fail || !(fail & nm)) continue;"),
    "flag_p3_dropped": ("                    lf |= FL_P3;\n", "                    ;\n"),
    "flag_margin_road_ignored": ("r->kchi = lmin > 0.0 ? 2.0 * sqrt(ey * ey + ez * ez) / sqrt(lmin) : INFINITY;",
                                 "r->kchi = 0.0;"),
    "flag_margin_largest_eigenvalue": ("const double lmin = 0.5 * (Syy + Szz) - sqrt(h * h + Syz * Syz);",
                                       "const double lmin = 0.5 * (Syy + Szz) + sqrt(h * h + Syz * Syz);"),
    "flag_p1_dropped": ("if (bnear) lf |= FL_P1;", ""),
}


PINS = ["test_oracle_math.py", "test_oracle_search.py", "test_oracle_beam.py", "test_oracle_refit.py",
        "test_oracle_residuals.py", "test_oracle_realistic.py", "test_oracle_resolution.py",
        "test_oracle_flags.py", "test_oracle_field.py"]


def _run_mutant(name, tmp):
    src = open(SRC).read()
    a, b = MUTANTS[name]
    if src.count(a) < 1:
        return "site"
    path = os.path.join(tmp, f"{name}.c")
    lib = os.path.join(tmp, f"{name}.so")
    with open(path, "w") as f:
        f.write(src.replace(a, b, 1))
    subprocess.run(["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-o", lib, path, "-lm"], check=True)
    env = dict(os.environ, TRD_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider"] +
                       [os.path.join(ROOT, "tests", p) for p in PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    return "caught" if r.returncode != 0 else "passed"


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    """Every planted mistake against the pin suite, several at a time."""
    tmp = str(tmp_path_factory.mktemp("mutants"))
    with ThreadPoolExecutor(max_workers=max(1, min(6, (os.cpu_count() or 2) - 1))) as ex:
        futs = {n: ex.submit(_run_mutant, n, tmp) for n in MUTANTS}
        return {n: f.result() for n, f in futs.items()}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, outcomes):
    assert outcomes[name] != "site", f"mutation site of {name} not found"
    assert outcomes[name] == "caught", f"planted mistake {name} passed every pin"
