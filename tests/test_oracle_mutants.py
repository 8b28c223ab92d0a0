"""The pins must catch plausible mistakes in the oracle.

Each case copies the oracle source, plants one mistake (a dropped term, a
wrong sign, a transposed operand, a wrong index), builds it into a temporary
library, swaps it in for the real one and checks that at least one pin fails.
Everything runs on the CPU; the real oracle is never modified.
"""
import ctypes
import os
import subprocess
import tempfile

import pytest

import oracle as O
from oracle import build as OB
from tests import test_oracle_dg as DG
from tests import test_oracle_pins as PINS
from tests import test_oracle_simplex as SX
from tests import test_oracle_stokes as ST
from tests import test_oracle_vector as VX

# the oracle's sources: fe_oracle.c includes the simplex part
ORACLE_FILES = ("fe_oracle.c", "fe_oracle_simplex.c")

MUTANTS = {
    "transposed_inverse_jacobian": ("g += Ji[s * dim + i] * gref[s];", "g += Ji[i * dim + s] * gref[s];"),
    "elasticity_mu_term_untransposed": ("+ mu * grad[a * dim + j] * grad[b * dim + i];",
                                        "+ mu * grad[a * dim + i] * grad[b * dim + j];"),
    "lifting_sign": ("else rhs[g[a]] -= A[a * nloc + b] * uD[b];", "else rhs[g[a]] += A[a * nloc + b] * uD[b];"),
    "dropped_quadrature_weight": ("double wd = w * fabs(qp.detJ) * coef;", "double wd = fabs(qp.detJ) * coef;"),
    "gauss_weight_scale": ("w[n - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp);",
                           "w[n - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);"),
    "lagrange_derivative_sign": ("dnum += prod;", "dnum -= prod;"),
    "local_node_axes_swapped": ("int ar[3] = {a % (k + 1), (a / (k + 1)) % (k + 1), a / ((k + 1) * (k + 1))};\n    int64_t N0",
                                "int ar[3] = {(a / (k + 1)) % (k + 1), a % (k + 1), a / ((k + 1) * (k + 1))};\n    int64_t N0"),
    "load_without_shape_function": ("f[a * ncomp + c] += wd * fc * phi[a];", "f[a * ncomp + c] += wd * fc;"),
    "cg_beta_inverted": ("double beta = rho_new / rho;", "double beta = rho / rho_new;"),
    "geometry_derivative_sign": ("if (r == s) g *= vr ? 1.0 : -1.0;", "if (r == s) g *= vr ? -1.0 : 1.0;"),
    "l2_error_without_sqrt": ("return sqrt(err2);", "return err2;"),
    "dg_mean_without_half": ("double v = -sg[i] * ph[i][a] * dnb * 0.5 - tau",
                             "double v = -sg[i] * ph[i][a] * dnb - tau"),
    "dg_boundary_normal_inward": ("n[i] = (side ? 1.0 : -1.0) * nv[i] / dS;  /* outward */",
                                  "n[i] = nv[i] / dS;  /* outward */"),
    "dg_penalty_not_scaled_by_facet_size": ("            double sigma = gamma / hF;\n            for (int q = 0; q < np; q++) {\n                double xK[3]",
                                            "            double sigma = gamma;\n            for (int q = 0; q < np; q++) {\n                double xK[3]"),
    "dg_boundary_load_tau_sign": ("rhs[K * nn + a] += W * (-tau * uD * dna", "rhs[K * nn + a] += W * (tau * uD * dna"),
    "l2_error_dropped_weight": ("err2 += w * fabs(qp.detJ) * (ue - uh) * (ue - uh);",
                                "err2 += fabs(qp.detJ) * (ue - uh) * (ue - uh);"),
    "stokes_divergence_sign": ("B[a * nlu + dim * b + c] -= wd * psi[a] * gu[b * dim + c];",
                               "B[a * nlu + dim * b + c] += wd * psi[a] * gu[b * dim + c];"),
    "stokes_dropped_jacobian": ("double wd = w * fabs(qu.detJ);\n        for (int a = 0; a < nnp; a++) {\n            md[a]",
                                "double wd = w;\n        for (int a = 0; a < nnp; a++) {\n            md[a]"),
    "stokes_wrong_velocity_component": ("wd * psi[a] * gu[b * dim + c];", "wd * psi[a] * gu[b * dim + (c + 1) % dim];"),
    "simplex_basis_untransposed": ("Phi[a * nn + b] = Ci[b * nn + a];", "Phi[a * nn + b] = Ci[a * nn + b];"),
    "simplex_collapsed_jacobian_power": ("jac = (1.0 - u0) * (1.0 - u0) * (1.0 - u1);", "jac = (1.0 - u0) * (1.0 - u1);"),
    "simplex_gradient_untransposed_jacobian": ("g += Ji[r * dim + i] * dref[a * dim + r];",
                                               "g += Ji[i * dim + r] * dref[a * dim + r];"),
    "simplex_barycentric_vertex_shift": ("lam[r + 1] = s[3 * a + r];", "lam[r + 1] = s[3 * a + (r + 1) % dim];"),
    "simplex_boundary_facet_vertex": ("lj = s[3 * a + j - 1];", "lj = s[3 * a + j % dim];"),
    "simplex_node_position_axis": ("(X[(t + 1) * dim + r] - X[r]) * s[3 * a + t] / k;",
                                   "(X[(t + 1) * dim + r] - X[r]) * s[3 * a + r] / k;"),
    "simplex_load_without_jacobian": ("double wd = qw[q] * fabs(det);\n        for (int c = 0; c < ncomp; c++) {\n            double fc",
                                      "double wd = qw[q];\n        for (int c = 0; c < ncomp; c++) {\n            double fc"),
    "simplex_lifting_sign": ("else rhs[g[i]] -= A[i * nloc + j] * ud[j];", "else rhs[g[i]] += A[i * nloc + j] * ud[j];"),
    "simplex_l2_error_without_sqrt": ("double norm = sqrt(err2);", "double norm = err2;"),
    "simplex_numbering_not_first_appearance": ("qsort(grp, ng, sizeof(sx_first), sx_first_cmp);", ""),
    "vector_edge_orientation_ignored": ("sgn[a] = g[i] < g[j] ? 1.0 : -1.0;", "sgn[a] = 1.0;"),
    "vector_facet_orientation_ignored": ("sgn[a] = (inv % 2) ? -1.0 : 1.0;", "sgn[a] = 1.0;"),
    "vector_covariant_map_untransposed": (
        "v += !vx_contra(family) ? Ji[r * dim + c] * phi[a * dim + r] : J[c * dim + r] * phi[a * dim + r] / det;",
        "v += !vx_contra(family) ? Ji[c * dim + r] * phi[a * dim + r] : J[c * dim + r] * phi[a * dim + r] / det;"),
    "vector_contravariant_map_without_det": (
        "v += !vx_contra(family) ? Ji[r * dim + c] * phi[a * dim + r] : J[c * dim + r] * phi[a * dim + r] / det;",
        "v += !vx_contra(family) ? Ji[r * dim + c] * phi[a * dim + r] : J[c * dim + r] * phi[a * dim + r];"),
    "vector_curl_map_without_det": ("Cp[a * 3 + c] = v / det;", "Cp[a * 3 + c] = v;"),
    "vector_edge_tangent_reversed": ("d += v[t] * (xj[t] - xi[t]);", "d += v[t] * (xi[t] - xj[t]);"),
    "vector_boundary_edge_test": ("on = i1 != j && j1 != j;", "on = i1 != j || j1 != j;"),
    "vector_mass_without_kappa": ("Al[a * nd + b] += wd * (coef * st + kappa * ms);", "Al[a * nd + b] += wd * (coef * st + ms);"),
    "nedelec2_edge_reversal_sign": ("T[a * nd + a + 1] = -1.0;", "T[a * nd + a + 1] = 1.0;"),
    "nedelec2_edge_weights_swapped": ("double qv = slot < 0 ? 1.0 : slot == 0 ? 1.0 - gx[q] : gx[q];",
                                      "double qv = slot < 0 ? 1.0 : slot == 0 ? gx[q] : 1.0 - gx[q];"),
    "nedelec2_face_block_transposed": ("T[(a + m) * nd + a + b] = P[m + 1][b] - P[0][b];",
                                       "T[(a + b) * nd + a + m] = P[m + 1][b] - P[0][b];"),
    "rt2_facet_parity_ignored": ("T[(f * dim + x) * nd + f * dim + rank[x]] = (inv % 2) ? -1.0 : 1.0;",
                                 "T[(f * dim + x) * nd + f * dim + rank[x]] = 1.0;"),
    "rt2_facet_vertex_order_ignored": ("T[(f * dim + x) * nd + f * dim + rank[x]] = (inv % 2) ? -1.0 : 1.0;",
                                       "T[(f * dim + x) * nd + f * dim + x] = (inv % 2) ? -1.0 : 1.0;"),
    "rt2_flux_weight_of_first_vertex": ("s += fw[q] * d * lam[k];", "s += fw[q] * d * lam[0];"),
    "rt2_interior_key_slot": ("slot = family == 3 ? a - 6 : a - dim * (dim + 1);", "slot = family == 3 ? a - 6 : 0;"),
    "l2_error_dropped_jacobian": ("err2 += w * fabs(qp.detJ) * (ue - uh) * (ue - uh);",
                                  "err2 += w * (ue - uh) * (ue - uh);"),
}

# the pins run against each mutant (small, fast parametrizations)
PIN_CALLS = [
    lambda: PINS.test_gauss_legendre_matches_numpy_and_is_exact(3),
    lambda: PINS.test_lagrange_delta_partition_and_exact_polynomials(2),
    lambda: PINS.test_paper_bicubic_quad_numbering(),
    lambda: PINS.test_poisson_element_affine_closed_form(3, 2),
    lambda: PINS.test_elasticity_element_affine_closed_form(3, 2),
    lambda: PINS.test_energy_of_linear_fields(),
    lambda: PINS.test_global_kernel_and_load_without_dirichlet(3, 1, "poisson"),
    lambda: PINS.test_linear_patch_test(2, 3, 3, "poisson"),
    lambda: PINS.test_linear_patch_test(3, 1, 3, "elasticity"),
    lambda: PINS.test_pcg_matches_direct_solve_and_lanczos_bounds(2, 2, "poisson"),
    lambda: PINS.test_l2_norm_of_sine_product_closed_form(2, 2, 6, 0.2),
    lambda: PINS.test_l2_norm_of_affine_field_is_exact(3, 1, 3, 0.2),
    lambda: PINS.test_l2_norm_of_vector_field_sums_components(),
    lambda: DG.test_dg_box_matrix_closed_form(2, [3, 2], 3, 1.0),
    lambda: DG.test_dg_linear_patch_test(2, [3, 4], 1),
    lambda: ST.test_b_element_box_closed_form(2, 2),
    lambda: ST.test_constant_force_is_balanced_by_an_affine_pressure(2, [3, 4], 1),
    lambda: SX.test_local_nodes_and_basis_match_silvester(2, 2),
    lambda: SX.test_collapsed_rule_integrates_monomials_exactly(3, 3),
    lambda: SX.test_poisson_element_matches_exact_reference_tensor(3, 2),
    lambda: SX.test_load_of_constant_source_is_exact_moment(3, 2),
    lambda: SX.test_numbering_matches_brute_force_by_position(3, 2, 2, True),
    lambda: SX.test_linear_patch_test(3, 1, "poisson", 3),
    lambda: SX.test_linear_patch_test(3, 2, "elasticity", 2),
    lambda: SX.test_l2_error_magnitude_closed_forms(2, 2),
    lambda: VX.test_shape_functions_are_whitney_forms("nedelec", 3),
    lambda: VX.test_shape_functions_are_whitney_forms("raviart_thomas", 3),
    lambda: VX.test_element_matrix_matches_exact_whitney_integrals("nedelec", 3),
    lambda: VX.test_element_matrix_matches_exact_whitney_integrals("raviart_thomas", 2),
    lambda: VX.test_curl_curl_annihilates_discrete_gradients(3),
    lambda: VX.test_div_div_annihilates_discrete_curls_3d(),
    lambda: VX.test_constant_field_patch_test("nedelec", 3),
    lambda: VX.test_constant_field_patch_test("raviart_thomas", 3),
    lambda: VX.test_l2_convergence_to_manufactured_field("nedelec", 2, (8, 16)),
    lambda: VX.test_nedelec2_interpolates_its_space_exactly(3),
    lambda: VX.test_nedelec2_linear_curl_free_patch_test(3, 2),
    lambda: VX.test_nedelec2_curl_curl_annihilates_gradients_of_p2(3, 2),
    lambda: VX.test_rt2_interpolates_its_space_exactly(3),
    lambda: VX.test_rt2_divergence_free_affine_patch_test(3, 2),
    lambda: VX.test_rt2_div_div_kernel_is_the_discrete_curls(3, [2, 1, 1]),
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, monkeypatch):
    old, new = MUTANTS[name]
    srcs = {f: open(os.path.join(os.path.dirname(OB.SRC), f)).read() for f in ORACLE_FILES}
    assert sum(s.count(old) for s in srcs.values()) == 1, "mutation site not found exactly once"
    with tempfile.TemporaryDirectory() as td:
        for f, s in srcs.items():
            with open(os.path.join(td, f), "w") as out:
                out.write(s.replace(old, new))
        path = os.path.join(td, "fe_oracle.c")
        so = os.path.join(td, "libmut.so")
        subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", so, path, "-lm"], check=True)
        real = O.lib()
        monkeypatch.setattr(O, "_lib", None)
        monkeypatch.setattr(OB, "LIB", so)
        O.lib()  # loads the mutant with the same argtypes
        caught = []
        for call in PIN_CALLS:
            try:
                call()
            except Exception:  # assertion or numerical failure both count
                caught.append(call)
        monkeypatch.setattr(O, "_lib", real)
        assert caught, f"no pin caught mutant {name}"
