"""The oracle's pins reject plausible mistakes.

Each case plants one mistake in a copy of oracle/oracle.c (a dropped factor,
a wrong sign or index, a transposed operand, a wrong tie-break order, a
missing normalisation), builds that copy with gcc into a temporary library
and runs the pin test that must reject it, in a child process that loads the
copy through ORACLE_LIB. The case passes when that pin test fails. Nothing
here touches the GPU path.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

INV = "tests/test_oracle_invariants.py::"
PIN = "tests/test_oracle_paper_pins.py::"
KC = "tests/test_oracle_kcycle.py::"
SW = "tests/test_oracle_smooth_w.py::"
CP = "tests/test_oracle_coarse_pcg.py::"
SM = "tests/test_oracle_smoothed.py::"

# (mistake, text in oracle.c, replacement, pin test that must reject it)
MUTATIONS = [
    ("eq. (weights): factor 2 dropped",
     "double num = ((2.0 * a) * w[i]) * w[j];", "double num = ((1.0 * a) * w[i]) * w[j];",
     INV + "test_weights_isotropic_closed_form"),
    ("eq. (weights): w_i for w_j in the denominator",
     "double den = (aii * w[i]) * w[i] + (ajj * w[j]) * w[j];",
     "double den = (aii * w[i]) * w[i] + (ajj * w[i]) * w[j];",
     INV + "test_weights_invariants"),
    ("eq. (weights): sign of the coupling term",
     "c[e] = 1.0 - num / den;", "c[e] = 1.0 + num / den;",
     PIN + "test_table1_gauss_seidel"),
    ("matching: lightest edges first",
     "if (a->c > b->c) return -1;\n  if (a->c < b->c) return 1;",
     "if (a->c < b->c) return -1;\n  if (a->c > b->c) return 1;",
     PIN + "test_table1_gauss_seidel"),
    ("matching: second tie-break reversed",
     "if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;\n  return 0;\n}\n\nint64_t",
     "if (a->hi != b->hi) return a->hi > b->hi ? -1 : 1;\n  return 0;\n}\n\nint64_t",
     INV + "test_matching_equals_locally_dominant"),
    ("matching: first tie-break reversed",
     "if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;\n  if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;\n  return 0;\n}\n\nint64_t",
     "if (a->lo != b->lo) return a->lo > b->lo ? -1 : 1;\n  if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;\n  return 0;\n}\n\nint64_t",
     INV + "test_tiny_exhaustive_matchings_on_path_graphs"),
    ("eq. (prolongator): norm without square root",
     "p[v] = w[v] / sqrt(s);", "p[v] = w[v] / s;",
     INV + "test_numbering_and_prolongator"),
    ("eq. (prolongator): singleton entry not normalised",
     "p[v] = w[v] / fabs(w[v]);", "p[v] = 1.0;",
     INV + "test_numbering_and_prolongator"),
    ("Galerkin product: p_lo for p_hi",
     "buf[cnt].t = (p[lo] * a) * p[hi];", "buf[cnt].t = (p[lo] * a) * p[lo];",
     INV + "test_galerkin_matches_dense_product"),
    ("restriction of w: prolongator weights dropped",
     "double t = p[i] * v[i];", "double t = v[i];",
     INV + "test_numbering_and_prolongator"),
    ("l1-Jacobi: absolute value dropped",
     "} else {\n        s = s + fabs(A->val[k]);", "} else {\n        s = s + A->val[k];",
     PIN + "test_table1_l1_jacobi"),
    ("l1-Jacobi: plain diagonal",
     "m[i] = aii + s;", "m[i] = aii;",
     PIN + "test_table1_l1_jacobi"),
    ("eq. (amg): post-smoothing sign",
     "for (int32_t i = 0; i < n; ++i) z[i] = z[i] + (r[i] - t[i]) / m[i];\n  }\n  free(t);",
     "for (int32_t i = 0; i < n; ++i) z[i] = z[i] - (r[i] - t[i]) / m[i];\n  }\n  free(t);",
     INV + "test_vcycle_two_level_equals_error_propagation_product"),
    ("eq. (amg): prolongation without P's values",
     "z[i] = z[i] + h->p[l][i] * zc[h->agg[l][i]];", "z[i] = z[i] + zc[h->agg[l][i]];",
     INV + "test_vcycle_two_level_equals_error_propagation_product"),
    ("eq. (amg): residual sign",
     "for (int32_t i = 0; i < n; ++i) t[i] = r[i] - t[i];",
     "for (int32_t i = 0; i < n; ++i) t[i] = r[i] + t[i];",
     INV + "test_vcycle_two_level_equals_error_propagation_product"),
    ("CG: beta inverted",
     "double beta = rz / rho;", "double beta = rho / rz;",
     INV + "test_pcg_small_case_against_dst_exact"),
    ("Cholesky: back substitution with L for its transpose",
     "for (int32_t k = i + 1; k < n; ++k) t = t - L[(int64_t)k * n + i] * z[k];",
     "for (int32_t k = i + 1; k < n; ++k) t = t - L[(int64_t)i * n + k] * z[k];",
     INV + "test_cholesky_against_lapack"),
    ("sweep composition: earlier prolongator dropped",
     "p_c[i] = p_c[i] * pk[a];", "p_c[i] = pk[a];",
     INV + "test_isotropic_hierarchy_closed_form"),
    ("numbering: partner of a pair left unnumbered",
     "if (mate[v] >= 0) agg[mate[v]] = next;", "if (mate[v] >= 0 && 0) agg[mate[v]] = next;",
     PIN + "test_table1_gauss_seidel"),
    ("K-cycle FCG: sign of the orthogonalisation term in rho2",
     "double rho2 = dot(n, c2, v2) - gamma * gamma / rho1;",
     "double rho2 = dot(n, c2, v2) + gamma * gamma / rho1;",
     KC + "test_fcg2_is_the_galerkin_projection"),
    ("K-cycle FCG: sign of the correction of the first coefficient",
     "double a1 = s1 - s2 * (gamma / rho1);", "double a1 = s1 + s2 * (gamma / rho1);",
     KC + "test_fcg2_is_the_galerkin_projection"),
    ("K-cycle FCG: second step length from b instead of r1",
     "double s2 = dot(n, c2, r1) / rho2;", "double s2 = dot(n, c2, b) / rho2;",
     KC + "test_fcg2_is_the_galerkin_projection"),
    ("outer FCG: sign of beta",
     "double beta = -dot(n, z, q) / pq;", "double beta = dot(n, z, q) / pq;",
     KC + "test_fcg_with_vcycle_equals_pcg"),
    ("smooth w: sweep with the wrong sign",
     "for (int32_t i = 0; i < n; ++i) w[i] = w[i] - t[i] / m[i];",
     "for (int32_t i = 0; i < n; ++i) w[i] = w[i] + t[i] / m[i];",
     SW + "test_every_sweep_lowers_the_energy"),
    ("K-cycle: coarse correction by the plain cycle (no FCG)",
     "if (kcycle && l + 1 < L) fcg2(h, l + 1, pre, post, rc, zc);",
     "if (0 && kcycle && l + 1 < L) fcg2(h, l + 1, pre, post, rc, zc);",
     KC + "test_kcycle_iterations_do_not_grow_with_the_grid"),
    ("coarsest CG: residual not preconditioned",
     "z[i] = r[i] / m[i]; /* preconditioned residual */",
     "z[i] = r[i]; /* preconditioned residual */",
     CP + "test_coarse_pcg_is_scipy_cg_with_the_l1_diagonal"),
    ("coarsest CG: beta inverted",
     "double beta = rz1 / rz0;", "double beta = rz0 / rz1;",
     CP + "test_coarse_pcg_terminates_at_the_exact_solution"),
    ("coarsest CG: stop test on the squared residual norm",
     "if (sqrt(dot(n, r, r)) < rtol * bnorm) break;",
     "if (dot(n, r, r) < rtol * bnorm) break;",
     CP + "test_coarse_pcg_is_scipy_cg_with_the_l1_diagonal"),
    ("coarsest CG: the hierarchy keeps the Cholesky solve",
     "if (h->coarse_solver == 1)", "if (h->coarse_solver == 7)",
     CP + "test_vcycle_with_iterative_coarsest_solves_the_coarsest_system"),
    ("smoothed P: tentative term dropped",
     "double base = J == agg[i] ? p[i] : 0.0;", "double base = 0.0;",
     SM + "test_pbar_is_the_dense_formula"),
    ("smoothed P: D^-1 dropped",
     "double t = acc[J] / aii;", "double t = acc[J];",
     SM + "test_pbar_is_the_dense_formula"),
    ("smoothed P: omega from the row sums without |.|",
     "for (int64_t k = A->rp[i]; k < A->rp[i + 1]; ++k) s = s + fabs(A->val[k]);\n    double r",
     "for (int64_t k = A->rp[i]; k < A->rp[i + 1]; ++k) s = s + A->val[k];\n    double r",
     SM + "test_omega_is_four_thirds_over_the_inf_norm_of_the_scaled_matrix"),
    ("smoothed P: omega = 1 / ||D^-1 A||_inf (the text's formula)",
     "  return 4.0 / (3.0 * nrm);", "  return 1.0 / nrm;",
     PIN + "test_supplement_smoothed_K_gauss_seidel"),
    ("general Galerkin: coefficient dropped in the row combination",
     "double t = coef[k] * B->val[e];", "double t = B->val[e];",
     SM + "test_galerkin_with_pbar_is_the_dense_product"),
    ("smoothed cycle: prolongation by the tentative P",
     "csr_apply(&h->Pb[l], zc, u); /* u = Pbar zc */",
     "for (int32_t i = 0; i < n; ++i) u[i] = h->p[l][i] * zc[h->agg[l][i]];",
     SM + "test_two_level_vcycle_is_the_error_propagation_product"),
]


def _run_mutant(case, workdir):
    name, old, new, pin = case
    src = open(SRC).read()
    if src.count(old) != 1:
        return "oracle.c no longer holds the text this case mutates"
    os.makedirs(workdir, exist_ok=True)
    mutant = os.path.join(workdir, "oracle.c")
    with open(mutant, "w") as f:
        f.write(src.replace(old, new, 1))
    lib = os.path.join(workdir, "liboracle.so")
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                    "-I", os.path.dirname(SRC), "-o", lib, mutant, "-lm"],
                   check=True, capture_output=True)
    env = dict(os.environ, ORACLE_LIB=lib, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1",
               MKL_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", pin],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    if r.returncode == 1:
        return None
    return "pin %s did not reject it (exit %d):\n%s" % (pin, r.returncode, r.stdout[-2000:])


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    """Every mutant built and checked once, four child processes at a time."""
    from concurrent.futures import ThreadPoolExecutor

    base = tmp_path_factory.mktemp("mutants")
    workers = max(1, min(4, (os.cpu_count() or 1) // 2))
    with ThreadPoolExecutor(workers) as ex:
        res = list(ex.map(lambda kc: _run_mutant(kc[1], str(base / str(kc[0]))),
                          enumerate(MUTATIONS)))
    return {m[0]: r for m, r in zip(MUTATIONS, res)}


@pytest.mark.slow
@pytest.mark.parametrize("name", [m[0] for m in MUTATIONS])
def test_pin_rejects_planted_mistake(outcomes, name):
    assert outcomes[name] is None, outcomes[name]
