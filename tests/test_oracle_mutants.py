"""The oracle's pins must fail when a plausible mistake is planted in the oracle.

Each case copies the oracle's C source, makes one small edit (a dropped dt, a
flipped sign, a wrong exponent or index, a non-conservative update), builds it
into a temporary library and runs the pin tests against it in a subprocess.
The pins pass on the real oracle (test_oracle_pins.py); here every mutant must
make at least one of them fail.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "flood_oracle.c")

MUTANTS = {
    "dt_dropped_from_gravity_term": ("double num = q - ((g * hf) * dt) * grad;",
                                     "double num = q - (g * hf) * grad;"),
    "gravity_sign_flipped": ("double num = q - ((g * hf) * dt) * grad;",
                             "double num = q + ((g * hf) * dt) * grad;"),
    "friction_exponent_4_3": ("/ ((hf * hf) * cbrt(hf));", "/ (hf * cbrt(hf));"),
    "hf_min_bed": ("double hf = fmax(etaL, etaR) - fmax(zL, zR);",
                   "double hf = fmax(etaL, etaR) - fmin(zL, zR);"),
    "face_roughness_one_sided": ("double nf = 0.5 * (nL + nR);", "double nf = nL;"),
    "boundary_exponent_2_3": ("return x * (c * c);", "return c * c;"),
    "depth_update_sign": ("h[j * nx + i] + (dt * ((qW - qE) + (qS - qN))) / dx;",
                          "h[j * nx + i] + (dt * ((qW - qE) + (qN - qS))) / dx;"),
    "y_faces_use_x_neighbour": (
        "int64_t L = (j - 1) * nx + i, R = j * nx + i;\n                    double *q = &qy[",
        "int64_t L = j * nx + i - (i > 0), R = j * nx + i;\n                    double *q = &qy["),
    "donor_wrong_cell": ("if (*q > 0.0 && i >= 1) *q *= r[j * nx + i - 1];",
                         "if (*q > 0.0 && i < nx) *q *= r[j * nx + i];"),
    "budget_uses_unscaled_outflow": ("clk->v_out += dt * dx * sum_out;",
                                     "clk->v_out += 1.0001 * dt * dx * sum_out;"),
    "cfl_uses_sqrt_h_not_gh": ("dt = fmin(p->dt_max, p->alpha * dx / sqrt(g * hmax));",
                               "dt = fmin(p->dt_max, p->alpha * dx / sqrt(hmax));"),
    "inflow_bisection_direction": (
        "pow53(mid - zc[c]);\n        F -= Q;\n        if (F < 0.0) lo = mid; else hi = mid;",
        "pow53(mid - zc[c]);\n        F -= Q;\n        if (F > 0.0) lo = mid; else hi = mid;"),
    "last_step_not_shortened": ("if (dt >= rem) { dt = rem; last = 1; }",
                                "if (dt >= rem) { last = 1; }"),
}


# Mistakes planted in the two method variants; their pins must catch them.
VAR_MUTANTS = {
    "vector_mean_rows_shifted": ("for (int64_t jj = j; jj <= j + 1; jj++) {",
                                 "for (int64_t jj = j - 1; jj <= j; jj++) {"),
    "vector_mean_columns_shifted": ("for (int64_t ii = i; ii <= i + 1; ii++) {",
                                    "for (int64_t ii = i - 1; ii <= i; ii++) {"),
    "vector_mean_counts_border_faces": ("if (jj < 1 || jj > ny - 1) continue;",
                                        "if (jj < 0 || jj > ny) continue;"),
    "vector_uses_own_component_only": ("sqrt(q * q + qp * qp), dx, dt, g, p->h_eps);\n            }\n            if",
                                       "fabs(q), dx, dt, g, p->h_eps);\n            }\n            if"),
    "cell_area_outflow_exponent_5_3": ("(p->boundary_cell_area ? dx * pow23(hc) : pow53(hc));",
                                       "(p->boundary_cell_area ? dx * pow53(hc) : pow53(hc));"),
    "cell_area_outflow_factor_dropped": ("(p->boundary_cell_area ? dx * pow23(hc) : pow53(hc));",
                                         "(p->boundary_cell_area ? pow23(hc) : pow53(hc));"),
    "cell_area_inflow_face_factor_dropped": ("q_out[c] = dx * kc[c] * pow23(W - zc[c]);",
                                             "q_out[c] = kc[c] * pow23(W - zc[c]);"),
    "cell_area_inflow_sum_one_dx": ("F += dx * (dx * kc[c] * pow23(mid - zc[c]));",
                                    "F += dx * kc[c] * pow23(mid - zc[c]);"),
    "cell_area_inflow_bisection_direction": (
        "pow23(mid - zc[c]));\n        F -= Q;\n        if (F < 0.0) lo = mid; else hi = mid;",
        "pow23(mid - zc[c]));\n        F -= Q;\n        if (F > 0.0) lo = mid; else hi = mid;"),
}


# Mistakes planted in the reverse-mode sweep; the finite-difference pins must catch them.
ADJ_SRC = os.path.join(ROOT, "oracle", "flood_oracle_adjoint.c")
ADJ_MUTANTS = {
    "adj_limiter_depth_term_dropped": (
        "lh[c] = lh1[c] + ((w->lim[c] && h[c] > 0.0) ? w->rho[c] / w->O[c] : 0.0);",
        "lh[c] = lh1[c];"),
    "adj_donor_scaling_ignored": ("w->mus[f] = w->mu[f] * rd + nud * sgn(w->qs[f]);",
                                  "w->mus[f] = w->mu[f];"),
    "adj_friction_partial_sign": ("*Pn = -qs * dden_dnf / den;", "*Pn = qs * dden_dnf / den;"),
    "adj_depth_coupling_sign": ("w->mu[f] = l1 + cdt * (hR - hL);", "w->mu[f] = l1 + cdt * (hL - hR);"),
    "adj_inflow_roughness_path_dropped": ("double dLdk = p53(W - zc[k]) * (a_in[k] - dx * A / D);",
                                          "double dLdk = p53(W - zc[k]) * a_in[k];"),
    "adj_hydrograph_weights_swapped": ("grad_q[k] += (1.0 - wgt) * dLdQ;",
                                       "grad_q[k] += wgt * dLdQ;"),
}


def _build_and_run_pins(tmp_path, src_path, old, new, pins, name):
    src = open(src_path).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mut = tmp_path / os.path.basename(src_path)
    mut.write_text(src.replace(old, new))
    other = [os.path.join(ROOT, "oracle", f) for f in ("flood_oracle.c", "flood_oracle_adjoint.c")
             if f != os.path.basename(src_path)]
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                    "-shared", "-I", os.path.join(ROOT, "oracle"), "-o", str(lib), str(mut), *other,
                    "-lm"], check=True)
    env = dict(os.environ, FLOOD_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                          "--timeout", "60", os.path.join(ROOT, "tests", pins)],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode != 0, f"mutant {name} survived the pins:\n{res.stdout[-2000:]}"


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    _build_and_run_pins(tmp_path, SRC, old, new, "test_oracle_pins.py", name)


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(VAR_MUTANTS))
def test_variant_pins_catch_mutant(name, tmp_path):
    old, new = VAR_MUTANTS[name]
    _build_and_run_pins(tmp_path, SRC, old, new, "test_oracle_variants.py", name)


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(ADJ_MUTANTS))
def test_adjoint_pins_catch_mutant(name, tmp_path):
    old, new = ADJ_MUTANTS[name]
    _build_and_run_pins(tmp_path, ADJ_SRC, old, new, "test_oracle_adjoint.py", name)


# Forward mistakes a single face exposes: the hand-worked two-cell steps alone must catch them.
FACE_MUTANTS = ["dt_dropped_from_gravity_term", "gravity_sign_flipped", "friction_exponent_4_3",
                "hf_min_bed", "face_roughness_one_sided", "depth_update_sign",
                "y_faces_use_x_neighbour", "donor_wrong_cell"]


@pytest.mark.slow
@pytest.mark.parametrize("name", FACE_MUTANTS)
def test_face_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    _build_and_run_pins(tmp_path, SRC, old, new, "test_oracle_face_pin.py", name)
