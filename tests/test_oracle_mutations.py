"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case swaps one oracle step for a plausible wrong version (a dropped term,
a wrong sign, index or exponent, a missing transpose or symmetrisation) and
checks that at least one pin in ``test_oracle`` then fails.
"""

import inspect
import textwrap

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import oracle.sa_amg as sa
import oracle.schur as schur
import problems
from tests import test_oracle as pins
from tests import test_schur_oracle as schur_pins


def _pins_fail(golden):
    """True when the worked-example or dense-solve pins reject the oracle."""
    pw = pins.load_golden(golden)
    checks = [
        lambda: pins.test_worked_example_setup(pw),
        lambda: pins.test_worked_example_vcycle(pw),
        lambda: pins.test_galerkin_symmetric_spd("diffusion"),
        lambda: pins.test_spai0_closed_form_poisson(),
        lambda: pins.test_aggregation_phase2_joins_lowest_index_neighbour(),
        lambda: pins.test_strength_symmetrised_for_nonsymmetric(),
        lambda: pins.test_filtered_matrix_lumps_weak_entries(),
        lambda: pins.test_whole_solve_vs_dense(*pins._tiny_cases()[-1]),
        lambda: pins.test_vcycle_operator_symmetric_spd_linear("spai0"),
        lambda: pins.test_chebyshev_residual_polynomial_closed_form(3),
        lambda: pins.test_gmres_minimal_residual_over_krylov_space(),
        lambda: pins.test_gmres_arnoldi_relation_and_orthonormal_basis(),
        lambda: pins.test_pcg_iterate_minimises_energy_error_over_krylov_space(),
        lambda: pins.test_bicgstab_residual_is_product_of_stabilising_and_bicg_polynomials(),
        lambda: pins.test_hierarchy_fp32_is_the_rounded_fp64_hierarchy(),
        lambda: pins.test_fp32_vcycle_single_level_is_the_fp64_solve_rounded_once(),
        lambda: pins.test_fp32_two_grid_closed_form_within_rounding_bound(),
    ]
    for chk in checks:
        try:
            chk()
        except (AssertionError, ValueError, np.linalg.LinAlgError, sa.Breakdown):
            return True
    return False


def _spai0_wrong_numerator(A):
    A = sa._as_csr(A)
    return A.diagonal() ** 2 / np.asarray(A.multiply(A).sum(axis=1)).ravel()


def _aggregate_highest_neighbour(S):
    n = S.shape[0]
    ptr, nbr = S.indptr.tolist(), S.indices.tolist()
    agg = [sa.UNAGGREGATED] * n
    cnt = 0
    for i in range(n):
        if ptr[i] == ptr[i + 1]:
            agg[i] = sa.ISOLATED
    for i in range(n):
        if agg[i] == sa.UNAGGREGATED and all(agg[j] == sa.UNAGGREGATED for j in nbr[ptr[i]:ptr[i + 1]]):
            agg[i] = cnt
            for j in nbr[ptr[i]:ptr[i + 1]]:
                agg[j] = cnt
            cnt += 1
    snap = list(agg)
    for i in range(n):
        if agg[i] == sa.UNAGGREGATED:
            for j in reversed(nbr[ptr[i]:ptr[i + 1]]):  # wrong: highest index
                if snap[j] >= 0:
                    agg[i] = snap[j]
                    break
    return np.array(agg, dtype=np.int64)


def _strength_not_symmetrised(A, eps):
    A = sa._as_csr(A)
    d = A.diagonal()
    rows = sa._row_of_entry(A)
    strong = (A.indices != rows) & (A.data ** 2 > eps * eps * np.abs(d[rows] * d[A.indices]))
    n = A.shape[0]
    S = sp.csr_matrix((np.ones(int(strong.sum()), dtype=np.int8), (rows[strong], A.indices[strong])),
                      shape=(n, n))
    S.sort_indices()
    return S


def _filter_drops_weak(A, S):
    A_F, d_F = _orig["filtered_matrix"](A, S)
    d = sa._as_csr(A).diagonal()
    return (A_F - sp.diags(d_F) + sp.diags(d)).tocsr(), d


def _vcycle_wrong_sign(h, f, level=0):
    lv = h.levels[level]
    if level == h.nlevels - 1:
        return sa.sla.lu_solve(h.lu, f)
    z = lv.m * f
    r = f - lv.A @ z
    z = z + lv.P @ _vcycle_wrong_sign(h, lv.R @ r, level + 1)
    return z - lv.m * (f - lv.A @ z)  # wrong sign in the post-sweep


def _vcycle_restrict_tentative(h, f, level=0):
    lv = h.levels[level]
    if level == h.nlevels - 1:
        return sa.sla.lu_solve(h.lu, f)
    z = lv.m * f
    r = f - lv.A @ z
    fc = sa.tentative_prolongator(lv.agg).T @ r  # wrong: restricts with P_hat^T
    z = z + lv.P @ _vcycle_restrict_tentative(h, fc, level + 1)
    return z + lv.m * (f - lv.A @ z)


def _chebyshev_wrong_recurrence(A, dinv, f, x, hi, lo, degree):
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    sigma = theta / delta
    r = f - A @ x
    rho = 1.0 / sigma
    d = dinv * r / theta
    for step in range(degree):
        x = x + d
        r = r - A @ d
        if step == degree - 1:
            break
        rho_new = 1.0 / (2.0 * sigma + rho)  # wrong sign
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * r)
        rho = rho_new
    return x, r


def _arnoldi_skips_last_vector(A, precond, V, j):
    z = precond(V[j])
    w = A @ z
    h = np.zeros(j + 1)
    for _ in range(2):
        c = np.array([float(V[i] @ w) for i in range(j + 1)])
        for i in range(j):  # wrong: v_j itself is not projected out
            w = w - c[i] * V[i]
        h = h + c
    return z, h, float(np.sqrt(w @ w)), w


def _one_edit(fn, old, new, module=sa):
    """``fn`` recompiled from its source with the single occurrence of ``old``
    replaced by ``new`` (names resolve in the oracle module's namespace)."""
    src = textwrap.dedent(inspect.getsource(fn))
    assert src.count(old) == 1, (fn.__name__, old)
    ns = dict(module.__dict__)
    exec(compile(src.replace(old, new), "<mutant of %s>" % fn.__name__, "exec"), ns)
    return ns[fn.__name__]


_orig = {"filtered_matrix": sa.filtered_matrix, "prolongator_damping": sa.prolongator_damping}


MUTATIONS = {
    "spai0_numerator": ("spai0_diagonal", _spai0_wrong_numerator),
    "damping_constant": ("prolongator_damping", lambda A_F, d_F, iso: 0.5 * _orig["prolongator_damping"](A_F, d_F, iso)),
    "phase2_highest": ("aggregate", _aggregate_highest_neighbour),
    "strength_unsymmetrised": ("strength_graph", _strength_not_symmetrised),
    "filter_drops_weak": ("filtered_matrix", _filter_drops_weak),
    "post_sweep_sign": ("vcycle", _vcycle_wrong_sign),
    "restriction_tentative": ("vcycle", _vcycle_restrict_tentative),
    "chebyshev_recurrence_sign": ("chebyshev_sweep", _chebyshev_wrong_recurrence),
    "arnoldi_skips_last_vector": ("arnoldi_cgs2", _arnoldi_skips_last_vector),
    "pcg_beta_scaled": ("pcg", _one_edit(sa.pcg, "beta = rho_new / rho", "beta = 0.9 * rho_new / rho")),
    "bicgstab_beta_without_alpha_omega": (
        "bicgstab", _one_edit(sa.bicgstab, "beta = (rho / rho_old) * (alpha / omega)", "beta = rho / rho_old")),
    "bicgstab_omega_over_s_s": (
        "bicgstab", _one_edit(sa.bicgstab, "omega = float(t @ s) / float(t @ t)", "omega = float(t @ s) / float(s @ s)")),
    "vcycle_fp32_coarse_lu_in_fp32": (
        "vcycle_fp32", _one_edit(
            sa.vcycle_fp32,
            "return sla.lu_solve(h.lu, f32.astype(np.float64)).astype(np.float32)",
            "return sla.lu_solve(sla.lu_factor(h.levels[-1].A.toarray().astype(np.float32)), f32)")),
    "hierarchy_fp32_keeps_A_fp64": ("hierarchy_fp32", _one_edit(sa.hierarchy_fp32, "A=lv.A.astype(np.float32)", "A=lv.A")),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch, golden_dir):
    import os

    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(sa, attr, fn)
    monkeypatch.setattr(oracle, attr, fn)
    assert _pins_fail(os.path.join(golden_dir, "pw_1d_laplacian.txt")), name


def test_pins_pass_unmutated(golden_dir):
    import os

    assert not _pins_fail(os.path.join(golden_dir, "pw_1d_laplacian.txt"))


# ---------------------------------------------------------------- field split

def _schur_pins_fail():
    checks = [
        schur_pins.test_exact_inner_solves_invert_the_system,
        schur_pins.test_schur_matrix_elementwise_definition,
        schur_pins.test_schur_matrix_stencil_on_the_stokes_grid,
        schur_pins.test_diagonal_velocity_solve_with_exact_schur_inverts_the_lumped_system,
    ]
    for chk in checks:
        try:
            chk()
        except (AssertionError, ValueError, np.linalg.LinAlgError):
            return True
    return False


SCHUR_MUTATIONS = {
    "pressure_rhs_sign": ("field_split_apply", _one_edit(
        schur.field_split_apply, "r_p - b.D @ u_star", "r_p + b.D @ u_star", schur)),
    "divergence_as_minus_gradient_transpose": ("field_split_apply", _one_edit(
        schur.field_split_apply, "r_p - b.D @ u_star", "r_p + b.G.T @ u_star", schur)),
    "no_velocity_correction": ("field_split_apply", _one_edit(
        schur.field_split_apply, "u = u_star - vel_solve(b.G @ p)", "u = u_star", schur)),
    "schur_plus_sign": ("schur_matrix", _one_edit(
        schur.schur_matrix, "b.S - Dk @ b.G", "b.S + Dk @ b.G", schur)),
    "schur_with_full_inverse": ("schur_matrix", _one_edit(
        schur.schur_matrix, "dinv = sp.diags(1.0 / b.K.diagonal())",
        "dinv = sp.csr_matrix(np.linalg.inv(b.K.toarray()))", schur)),
    "schur_with_row_sums": ("schur_matrix", _one_edit(
        schur.schur_matrix, "dinv = sp.diags(1.0 / b.K.diagonal())",
        "dinv = sp.diags(1.0 / np.asarray(abs(b.K).sum(axis=1)).ravel())", schur)),
}


@pytest.mark.parametrize("name", sorted(SCHUR_MUTATIONS))
def test_planted_field_split_mistake_is_caught(name, monkeypatch):
    attr, fn = SCHUR_MUTATIONS[name]
    monkeypatch.setattr(schur, attr, fn)
    assert _schur_pins_fail(), name


def test_field_split_pins_pass_unmutated():
    assert not _schur_pins_fail()
