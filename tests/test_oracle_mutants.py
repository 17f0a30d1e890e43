"""The pins must catch plausible mistakes in the oracle.

Each case copies the oracle's C source, plants one mistake (a dropped term, a
wrong sign, a transposed index, a wrong colour, a misplaced weight, a wrong
sweep order, a nonzero cost term, a wrong multigrid transfer), compiles the
copy on the CPU and runs the pin suites against it.  They have to fail.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "colsten_oracle.c")

MUTANTS = {
    "dropped_corner_weight": (
        "    if (nnz == 2) return -1.0 / 6.0;\n    return -1.0 / 12.0;\n}",
        "    if (nnz == 2) return -1.0 / 6.0;\n    return 0.0;\n}"),
    "nonzero_q1_face": (
        "    if (nnz == 0) return 8.0 / 3.0;\n    if (nnz == 1) return 0.0;",
        "    if (nnz == 0) return 8.0 / 3.0;\n    if (nnz == 1) return -1.0 / 12.0;"),
    "sign_of_neighbour_sum": (
        "acc = fma(w, u[q + oz * g->sz + oy * g->sy + ox], acc);",
        "acc = fma(-w, u[q + oz * g->sz + oy * g->sy + ox], acc);"),
    "transposed_strides": (
        "return (g->dim == 3 ? k * g->sz : 0) + j * g->sy + i;",
        "return (g->dim == 3 ? k * g->sy : 0) + j * g->sz + i;"),
    "swapped_update_operands": (
        "    u[q] = og_over_centre(g->stencil, g->dim, rhs - acc);\n}",
        "    u[q] = og_over_centre(g->stencil, g->dim, acc - rhs);\n}"),
    "wrong_q1_centre": (
        "    if (stencil == 1) return x * 0.375;\n    return x / (2.0 * dim);",
        "    if (stencil == 1) return x / 3.0;\n    return x / (2.0 * dim);"),
    "dropped_plus_x_neighbour": (
        "            for (int ox = -1; ox <= 1; ++ox) {\n                if (ox == 0 && oy == 0 && oz == 0) continue;\n                double w",
        "            for (int ox = -1; ox <= 0; ++ox) {\n                if (ox == 0 && oy == 0 && oz == 0) continue;\n                double w"),
    "wrong_red_black_parity": (
        "int64_t s = (i - 1) + (j - 1) +",
        "int64_t s = (i - 1) + j +"),
    "q1_colour_axis_mixup": (
        "c |= (int)((j - 1 + parity) & 1) << 1;",
        "c |= (int)((i - 1 + parity) & 1) << 1;"),
    "jacobi_weight_dropped": (
        "dst[q] = fma(omega, og_over_centre(stencil, dim, h2 * b[q] - su), src[q]);",
        "dst[q] = og_over_centre(stencil, dim, h2 * b[q] - su) + src[q];"),
    "residual_scaled_wrongly": (
        "double rq = b[q] - su / h2;\n                if (r) r[q] = rq;",
        "double rq = b[q] - su * h2;\n                if (r) r[q] = rq;"),
    "neumaier_compensation_sign": (
        "if (fabs(*s) >= fabs(x)) *c += (*s - t) + x;",
        "if (fabs(*s) >= fabs(x)) *c += (t - *s) + x;"),
    "lex_sweep_reversed_x": (
        "                for (int64_t i = 1; i <= g.nx; ++i)\n                    og_update(&g, u, b, og_index(&g, i, j, k));",
        "                for (int64_t i = g.nx; i >= 1; --i)\n                    og_update(&g, u, b, og_index(&g, i, j, k));"),
    "cost_terms_not_zero": (
        "s = s + z * sin(",
        "s = s + (z + 1e-3) * sin("),
    "restrict_centre_weight": (
        "static double og_fw(int o) { return o == 0 ? 0.5 : 0.25; }",
        "static double og_fw(int o) { return o == 0 ? 0.25 : 0.25; }"),
    "restrict_shifted_block": (
        "int64_t qf = (dim == 3 ? 2 * K * szf : 0) + 2 * J * syf + 2 * I;",
        "int64_t qf = (dim == 3 ? 2 * K * szf : 0) + 2 * J * syf + 2 * I + 1;"),
    "restrict_keeps_coarse_guess": (
        "                bc[qc] = acc;\n                uc[qc] = 0.0;",
        "                bc[qc] = acc;"),
    "prolong_odd_weight": (
        "wx = (i & 1) ? 0.5 : 1.0;",
        "wx = (i & 1) ? 0.25 : 1.0;"),
    "prolong_wrong_coarse_index": (
        "(j / 2 + bb) * syc + i / 2 + c;",
        "(j / 2 + bb) * syc + (i + 1) / 2 + c;"),
    "correction_subtracted": (
        "uf[q] = uf[q] + acc;",
        "uf[q] = uf[q] - acc;"),
    "nd_cut_shifted": (
        "            m[a] = lo[a] + ext / 2;",
        "            m[a] = lo[a] + (ext - 1) / 2;"),
    "nd_leaves_skipped": (
        "                if (!any || on_cut) og_update(g, u, b, og_index(g, i, j, k));",
        "                if (on_cut) og_update(g, u, b, og_index(g, i, j, k));"),
    "fp32_jacobi_weight_dropped": (
        "dst[q] = fmaf(om, og_over_centre_f32(stencil, dim, h2 * b[q] - su), src[q]);",
        "dst[q] = og_over_centre_f32(stencil, dim, h2 * b[q] - su) + src[q];"),
    "fp32_lex_sweep_reversed_x": (
        "                for (int64_t i = 1; i <= g.nx; ++i)\n                    og_update_f32(&g, u, b, og_index(&g, i, j, k));",
        "                for (int64_t i = g.nx; i >= 1; --i)\n                    og_update_f32(&g, u, b, og_index(&g, i, j, k));"),
    "fp32_grid_residual_scaled_wrongly": (
        "                double rq = bq - su / h2;",
        "                double rq = bq - su * h2;"),
    "fp32_neighbour_term_dropped": (
        "                if (w == 0.0f) continue;\n                acc = fmaf(w, u[q + oz * g->sz + oy * g->sy + ox], acc);",
        "                if (w == 0.0f || (oy == 1 && oz == 0)) continue;\n                acc = fmaf(w, u[q + oz * g->sz + oy * g->sy + ox], acc);"),
    "gs_skips_last_colour": (
        "        for (int c = 0; c < nc; ++c)\n            og_colour_pass_f64(",
        "        for (int c = 0; c < nc - 1; ++c)\n            og_colour_pass_f64("),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation site not found: %s" % name
    mutated = src.replace(old, new, 1)
    csrc = tmp_path / "mutant.c"
    csrc.write_text(mutated)
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                    "-o", str(lib), str(csrc), "-lm"], check=True)
    env = dict(os.environ, COLSTEN_ORACLE_LIB=str(lib))
    proc = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                           os.path.join(ROOT, "tests", "test_oracle_fp32_pins.py"),
                           os.path.join(ROOT, "tests", "test_oracle_cost.py"),
                           os.path.join(ROOT, "tests", "test_oracle_mg.py"),
                           os.path.join(ROOT, "tests", "test_oracle_nd.py")],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert proc.returncode != 0, "the pins accepted mutant %s:\n%s" % (name, proc.stdout[-2000:])
