"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of oracle.cpp (a dropped or repeated
term, a wrong sign, weight, index or colouring), builds it on the CPU and runs
the pin suite against it in a subprocess: the suite must fail.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.cpp")

MUTANTS = {
    "dropped_neighbour_2d": ("const T s = (u[p - sx] + u[p + sx]) + (u[p - sy] + u[p + sy]);",
                             "const T s = (u[p - sx] + u[p + sx]) + (u[p - sy] + u[p - sy]);"),
    "stencil_sign_3d": ("return g.c * (T(6) * uC - s);", "return g.c * (T(6) * uC + s);"),
    "diag_2d": ("return g.c * (T(4) * uC - s);", "return g.c * (T(5) * uC - s);"),
    "smoother_sign": ("return u[p] + g.wd * r;", "return u[p] - g.wd * r;"),
    "colouring_3d": ("if (((i + j + k) & 1) != colour) continue; /* k = 0 in 2D */",
                     "if (((i + j) & 1) != colour) continue;"),
    "fw_edge_weight_2d": ("fc[q] = (T(0.25) * r[p] + T(0.125) * edges) + T(0.0625) * corners;",
                          "fc[q] = (T(0.25) * r[p] + T(0.25) * edges) + T(0.0625) * corners;"),
    "fw_index_3d": ("const T exz = (r[p - sx - sz] + r[p + sx - sz]) + (r[p - sx + sz] + r[p + sx + sz]);",
                    "const T exz = (r[p - sx - sy] + r[p + sx - sz]) + (r[p - sx + sz] + r[p + sx + sz]);"),
    "interp_edge": ("if (m == 1) return T(0.5) * (e[q] + e[q + s[0]]);", "if (m == 1) return T(0.5) * (e[q] + e[q]);"),
    "interp_cell_3d": ("((e[q + s[2]] + e[q + s[0] + s[2]]) + (e[q + s[1] + s[2]] + e[q + s[0] + s[1] + s[2]])));",
                       "((e[q + s[2]] + e[q + s[0] + s[2]]) + (e[q + s[1] + s[2]] + e[q + s[0] + s[1]])));"),
    "no_correction": ("u[p] = u[p] + interp_at(dim, nc, ec, i, j, k);", "u[p] = u[p];"),
    "kface_arith_mean": ("return ((T(2) * a) * b) / (a + b);", "return (a + b) / T(2);"),
    "varcoef_face_index": ("const T kyS = kface(k[p - sy], kp), kyC = kface(kp, k[p + sy]);",
                           "const T kyS = kface(k[p - sx], kp), kyC = kface(kp, k[p + sy]);"),
    "coarsest_diag": ("diag = g.c * (g.dim == 2 ? T(4) : T(6));", "diag = g.c * (g.dim == 2 ? T(4) : T(4));"),
    "jacobi_in_place": ("tmp[p] = smooth_at(g, u, f, p);", "u[p] = smooth_at(g, u, f, p); tmp[p] = u[p];"),
    "norm_skips_last_row": ("for (int j = 1; j < n - 1; ++j)\n            for (int i = 1; i < n - 1; ++i) {\n"
                            "                const double r = (double)residual_at",
                            "for (int j = 1; j < n - 2; ++j)\n            for (int i = 1; i < n - 1; ++i) {\n"
                            "                const double r = (double)residual_at"),
    "norm_no_sqrt": ("for (int k = k0; k < k1; ++k) s += part[(size_t)k];\n    return std::sqrt(s);",
                     "for (int k = k0; k < k1; ++k) s += part[(size_t)k];\n    return s;"),
    "norm_abs_not_square": ("s += r * r;", "s += std::fabs(r);"),
    "norm_plain_sum": ("s += r * r;", "s += r;"),
    "symmetric_post_red_first": ("rbgs_sweep(g, u, f, post);", "rbgs_sweep(g, u, f, 0);"),
    "w_cycle_restarts_from_zero": ("        mgcycle(H, l + 1, uc, fc, CYCLE_W);\n        mgcycle(H, l + 1, uc, fc, CYCLE_W);",
                                   "        mgcycle(H, l + 1, uc, fc, CYCLE_W);\n"
                                   "        std::fill(H.u[(size_t)l + 1].begin(), H.u[(size_t)l + 1].end(), T(0));\n"
                                   "        mgcycle(H, l + 1, uc, fc, CYCLE_W);"),
    "f_cycle_second_call_f": ("        mgcycle(H, l + 1, uc, fc, CYCLE_V);\n    }\n    prolong_correct",
                              "        mgcycle(H, l + 1, uc, fc, CYCLE_F);\n    }\n    prolong_correct"),
    "cg_beta_sign": ("p[x] = r[x] + beta * p[x];", "p[x] = r[x] - beta * p[x];"),
    "cg_alpha_inverted": ("const T alpha = (T)(rr / pq);", "const T alpha = (T)(pq / rr);"),
    "cg_residual_not_updated": ("r[x] = r[x] - alpha * q[x];", "r[x] = r[x];"),
    "half_rounds_toward_zero": ("double q = std::nearbyint(std::ldexp(a, 10 - E));",
                                "double q = std::trunc(std::ldexp(a, 10 - E));"),
    "half_subnormal_quantum": ("(uint16_t)std::nearbyint(std::ldexp(a, 24))", "(uint16_t)std::nearbyint(std::ldexp(a, 23))"),
    "fp16_scale_off_by_one": ("std::max(-126, 4 - e)", "std::max(-126, 5 - e)"),
    "fp16_correction_not_unscaled": ("u[p] = u[p] + (double)half_to_float(e16[p]) * inv;",
                                     "u[p] = u[p] + (double)half_to_float(e16[p]);"),
    "fp16_residual_not_scaled": ("r16[p] = float_to_half(s32 * (float)r[p]);", "r16[p] = float_to_half((float)r[p]);"),
    "cc_ghost_zero": ("const double uW = i > 0 ? u[p - 1] : uC, uE = i < n - 1 ? u[p + 1] : uC;",
                      "const double uW = i > 0 ? u[p - 1] : 0.0, uE = i < n - 1 ? u[p + 1] : uC;"),
    "cc_diagonal_not_reduced": ("L.wd[m] = (omega * (h * h)) / (double)(2 * dim - m);",
                                "L.wd[m] = (omega * (h * h)) / (double)(2 * dim);"),
    "cc_restrict_3d_weight": ("fc[cc_at(dim, nc, I, J, K)] = 0.125 * (q0 + q1);",
                              "fc[cc_at(dim, nc, I, J, K)] = 0.25 * (q0 + q1);"),
    "cc_prolong_transposed": ("u[p] = u[p] + ec[cc_at(dim, nc, i / 2, j / 2, dim == 3 ? k / 2 : 0)];",
                              "u[p] = u[p] + ec[cc_at(dim, nc, j / 2, i / 2, dim == 3 ? k / 2 : 0)];"),
    "cc_rhs_mean_kept": ("    cc_remove_mean(dim, n, fh.data());\n", ""),
    "cd_face_not_averaged": ("*gf = Cx{0.5 * (gp.re + gq.re), 0.5 * (gp.im + gq.im)};", "*gf = gp;"),
    "cd_g_square_dropped": ("const double q = 1.0 / (1.0 + s * s);", "const double q = 1.0 / (1.0 + s);"),
    "cd_diag_without_time_term": ("const Cx D{P.itau + c * S.re, c * S.im};", "const Cx D{c * S.re, c * S.im};"),
    "cd_fas_coarse_rhs_linear": ("fc[q] = cx_add(cd_apply(P, nc, cc, uh, gc.data(), i, j, k), rc[(size_t)q]);",
                                 "fc[q] = rc[(size_t)q];"),
    "cd_correction_not_differenced": ("u[p] = cx_add(u[p], cx_sub(uc[q], uh[q]));", "u[p] = cx_add(u[p], uc[q]);"),
    "cd_complex_product_sign": ("return Cx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};",
                                "return Cx{a.re * b.re + a.im * b.im, a.re * b.im + a.im * b.re};"),
    "st_west_east_swapped": ("T t = (a[1] * u[p - sx] + a[2] * u[p + sx])", "T t = (a[2] * u[p - sx] + a[1] * u[p + sx])"),
    "st_bottom_top_swapped": ("t = t + (a[5] * u[p - sz] + a[6] * u[p + sz]);",
                              "t = t + (a[6] * u[p - sz] + a[5] * u[p + sz]);"),
    "st_weight_laplacian_diagonal": ("return (omega * (h * h)) / s0;", "return (omega * (h * h)) / 4.0;"),
    "st_coarsest_laplacian_diagonal": ("diag = g.c * g.st[0];", "diag = g.c * (g.dim == 2 ? T(4) : T(6));"),
    "cc_sum_skips_last_cell": ("for (int i = 0; i < n; ++i) row += u[cc_at(dim, n, i, j, k)];",
                               "for (int i = 0; i < n - 1; ++i) row += u[cc_at(dim, n, i, j, k)];"),
}

PIN_FILES = ["test_oracle_pins.py", "test_oracle_pins_variants.py", "test_oracle_pins_fp16.py",
             "test_oracle_pins_cc.py", "test_oracle_pins_cd.py", "test_oracle_pins_stencil.py"]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    """Only the pin suites run against the mutant: the golden histories, which
    the oracle itself wrote, take no part in catching it."""
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    mut = tmp_path / "oracle_mut.cpp"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "liboracle_mut.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                    str(mut), "-o", str(lib)], check=True)
    env = dict(os.environ, MG_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          *[os.path.join(ROOT, "tests", f) for f in PIN_FILES]],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode != 0, f"pins did not catch mutant {name}:\n{res.stdout[-2000:]}"
