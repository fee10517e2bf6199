"""The oracle's pins are sensitive: each plausible mistake, planted into the oracle on the
CPU, makes at least one pin fail."""
import inspect
import textwrap

import numpy as np
import pytest

from oracle import gsi_oracle as O
from tests import test_oracle as T

def _pins():
    return [
        lambda: T.test_rational_model_equals_direct_objective(True),
        lambda: T.test_rational_model_equals_direct_objective(False),
        T.test_retraction_is_polar_factor_and_orthonormal,
        lambda: T.test_derivative_matches_finite_differences(True),
        lambda: T.test_derivative_matches_finite_differences(False),
        T.test_derivative_at_zero_is_minus_gradient_norm_and_trace_zeta,
        T.test_branch_roots_stable_equal_naive_and_bracket,
        T.test_get_mu_p1_equals_two_by_two_rayleigh_ritz,
        T.test_get_mu_is_minimiser_on_a_scan,
        T.test_c1_rcg_matches_closed_form,
    ]


def _some_pin_fails():
    for pin in _pins():
        try:
            pin()
        except Exception:
            return True
    return False


def _dphi_no_square(mu, alpha, beta, gamma, zeta):
    num = zeta + (gamma - alpha * beta) * mu - beta * zeta * mu * mu
    return -float(np.sum(num / (1.0 + beta * mu * mu)))


def _roots_wrong_branch(alpha, beta, gamma, zeta):
    d = gamma - alpha * beta
    s = np.sqrt(d * d + 4.0 * beta * zeta * zeta)
    return np.where(d < 0.0, 2.0 * zeta / (-np.abs(d) + s + 1e-300) * 0.5, (d + s) / (2.0 * beta * zeta))


def _diagonals_zeta_sign(C, S, PtZ, PtY):
    b, V, a, g, z = ORIG["linesearch_diagonals"](C, S, PtZ, PtY)
    return b, V, a, g, -z


def _retraction_no_vt(X, P, mu, b, V):
    M = V * (1.0 / np.sqrt(1.0 + mu * mu * b))
    return (X - mu * P) @ M, M


def _gradient_sign(X, Y):
    G, C = ORIG["gradient"](X, Y)
    return -G, C


def _phi_model_gamma_dropped(mu, alpha, beta, gamma, zeta):
    return -0.5 * float(np.sum((alpha + 2.0 * zeta * mu) / (1.0 + beta * mu * mu)))


ORIG = {name: getattr(O, name) for name in
        ["dphi_model", "branch_roots", "linesearch_diagonals", "retraction", "gradient", "phi_model"]}

MUTATIONS = {
    "dphi_model": _dphi_no_square,
    "branch_roots": _roots_wrong_branch,
    "linesearch_diagonals": _diagonals_zeta_sign,
    "retraction": _retraction_no_vt,
    "gradient": _gradient_sign,
    "phi_model": _phi_model_gamma_dropped,
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(monkeypatch, name):
    monkeypatch.setattr(O, name, MUTATIONS[name])
    assert _some_pin_fails(), f"no pin caught a planted mistake in {name}"


# ---- the filter, tracking, stencil and Hermitian parts of the oracle: each mistake is
# planted by an exact one-place edit of the function's source, and must fail one of the
# pins written for that part


def _source_mutant(fn, old, new):
    src = textwrap.dedent(inspect.getsource(fn))
    assert src.count(old) == 1, (fn.__name__, old)
    ns = {}
    exec(compile(src.replace(old, new), f"<planted mistake in {fn.__name__}>", "exec"), fn.__globals__, ns)
    return ns[fn.__name__]


_CHEB_PINS = [lambda: T.test_chebyshev_filter_is_the_scaled_polynomial(-1.0, 1.0),
              lambda: T.test_chebyshev_filter_is_the_scaled_polynomial(-0.5, 1.5),
              T.test_chebyshev_si_matches_brute_force_and_needs_fewer_products]
_HERM_PINS = [T.test_hermitian_rcg_magnetic_ring_closed_form, T.test_hermitian_rcg_dense_random_matches_library_eigh,
              T.test_hermitian_rcg_on_a_real_matrix_follows_the_real_iteration]

SOURCE_MUTATIONS = {
    "chebyshev: sign of the normalization recurrence": (
        "chebyshev_filter", "sigma_new = 1.0 / (2.0 / sigma1 - sigma)", "sigma_new = 1.0 / (2.0 / sigma1 + sigma)",
        _CHEB_PINS),
    "chebyshev: shift dropped in the recurrence": (
        "chebyshev_filter", "(A_op @ cur - c * cur)", "(A_op @ cur)", _CHEB_PINS),
    "chebyshev: first step unshifted": (
        "chebyshev_filter", "cur = (sigma1 / h) * (Y - c * X)", "cur = (sigma1 / h) * Y", _CHEB_PINS),
    "rcg: restart period off by one": (
        "rcg", "(k_restart > 0 and k % k_restart == 0)", "(k_restart > 0 and k % (k_restart + 1) == 0)",
        [T.test_restart_every_step_is_steepest_descent]),
    "rcg: Fletcher-Reeves instead of Polak-Ribiere": (
        "rcg", "beta_pr = (gg - float(np.sum(G_old * G))) / den", "beta_pr = gg / den",
        [T.test_hermitian_rcg_on_a_real_matrix_follows_the_real_iteration]),
    "rcg: conjugate direction not projected onto the tangent space": (
        "rcg", "P = tangent(X, G + beta_pr * P_old)", "P = G + beta_pr * P_old", [T.test_c1_rcg_matches_closed_form]),
    "rcg: sqrt(p) dropped from rho": (
        "rcg", "rho = np.sqrt(gg) / (np.sqrt(p) * nA)", "rho = np.sqrt(gg) / nA",
        [T.test_c1_rsd_matches_closed_form_and_invariants]),
    "norm: column sums instead of row sums": (
        "norm_inf", "float(abs(A).sum(axis=1).max())", "float(abs(A).sum(axis=0).max())",
        [T.test_norm_inf_is_the_library_matrix_infinity_norm]),
    "Rayleigh-Ritz: residuals paired with the reversed Ritz values": (
        "rayleigh_ritz", "R = AX @ U - V * w", "R = AX @ U - V * w[::-1]", [T.test_rayleigh_ritz_on_an_invariant_subspace]),
    "Cholesky QR: a single pass": ("cholesky_qr2", "for _ in range(2):", "for _ in range(1):", [T.test_cholesky_qr2]),
    "SplitMix64: second shift 28 instead of 27": (
        "splitmix64", "z = (z ^ (z >> np.uint64(27)))", "z = (z ^ (z >> np.uint64(28)))",
        [T.test_splitmix64_published_outputs]),
    "Box-Muller: the factor 2 under the square root dropped": (
        "seeded_start_block", "np.sqrt(-2.0 * np.log(u1))", "np.sqrt(-np.log(u1))",
        [T.test_seeded_start_block_is_standard_normal]),
    "Cholesky QR: lower factor used as the upper one": (
        "cholesky_qr2", "R = np.linalg.cholesky(sym(X.T @ X)).T", "R = np.linalg.cholesky(sym(X.T @ X))",
        [T.test_cholesky_qr2]),
    "principal angles: arccos of the cosines only": (
        "principal_angles", "return np.arctan2(s, c)", "return np.arccos(np.minimum(c[::-1], 1.0))",
        [T.test_cholesky_qr2, T.test_shift_invariance_and_basis_equivariance]),
    "tangent projector: wrong sign": (
        "tangent", "return D - X @ (X.T @ D)", "return D + X @ (X.T @ D)", [T.test_c1_rcg_matches_closed_form]),
    "line search: gamma from P^T A X": (
        "linesearch_diagonals", 'gamma = np.einsum("ki,kl,li->i", V, sym(PtZ), V)',
        'gamma = np.einsum("ki,kl,li->i", V, sym(PtY), V)', [T.test_get_mu_p1_equals_two_by_two_rayleigh_ritz]),
    "line search: alpha from P^T P": (
        "linesearch_diagonals", 'alpha = np.einsum("ki,kl,li->i", V, C, V)',
        'alpha = np.einsum("ki,kl,li->i", V, sym(S), V)', [T.test_get_mu_p1_equals_two_by_two_rayleigh_ritz]),
    "Get_Mu: bracket at the last sign change": (
        "get_mu", "            break\n        lo = float(c)", "        lo = float(c)", [T.test_get_mu_is_minimiser_on_a_scan]),
    "Get_Mu: descent test at 0 flipped": ("get_mu", "if f(0.0) >= 0.0:", "if f(0.0) <= 0.0:",
                                          [T.test_get_mu_is_minimiser_on_a_scan]),
    "Get_Mu: bracket widened by halving": (
        "get_mu", "c = 2.0 * (lo if lo > 0.0 else 1.0)", "c = 0.5 * (lo if lo > 0.0 else 1.0)",
        [T.test_get_mu_p1_equals_two_by_two_rayleigh_ritz]),
    "retraction: no square root in D_mu": (
        "retraction", "M = (V * (1.0 / np.sqrt(1.0 + mu * mu * b))) @ V.T", "M = (V * (1.0 / (1.0 + mu * mu * b))) @ V.T",
        [T.test_retraction_is_polar_factor_and_orthonormal]),
    "retraction: step taken along +P": (
        "retraction", "return (X - mu * P) @ M, M", "return (X + mu * P) @ M, M", [T.test_c1_rcg_matches_closed_form]),
    "SI: the Rayleigh-Ritz product not counted": (
        "subspace_iteration", "        AQ = A_op @ Q\n        res.spmm += 1", "        AQ = A_op @ Q",
        [T.test_block_product_counts_are_the_products_made]),
    "Chebyshev SI: filter products counted as degree": (
        "chebyshev_si", "res.spmm += degree - 1", "res.spmm += degree", [T.test_block_product_counts_are_the_products_made]),
    "Chebyshev SI: A X not rotated with the Ritz vectors": (
        "chebyshev_si", "Y = AQ @ U", "Y = AQ", _CHEB_PINS),
    "tracking: every matrix restarted from X0": (
        "track", "X = r.X", "X = X", [T.test_track_restarts_from_previous_subspace]),
    "stencil: y neighbour at ny instead of nx": (
        "stencil_matrix", "(j < ny - 1, nx)", "(j < ny - 1, ny)", [T.test_stencil_matrix_spectrum_is_the_closed_form]),
    "stencil: opposite signs on the two sides of a bond": (
        "stencil_matrix", "vals += [np.full(a.size, float(off))] * 2",
        "vals += [np.full(a.size, float(off)), np.full(a.size, -float(off))]",
        [T.test_stencil_matrix_spectrum_is_the_closed_form]),
    "hermitian: transpose without conjugation in C": (
        "rcg_hermitian", "C = herm(X.conj().T @ Y)", "C = herm(X.T @ Y)", _HERM_PINS),
    "hermitian: transpose without conjugation in the tangent projector": (
        "rcg_hermitian", "tang = lambda D: D - X @ (X.conj().T @ D)", "tang = lambda D: D - X @ (X.T @ D)",
        _HERM_PINS),
    "hermitian: sign of zeta": (
        "rcg_hermitian", "zeta = -np.real(np.diag(VH @ (P.conj().T @ Y) @ V))",
        "zeta = np.real(np.diag(VH @ (P.conj().T @ Y) @ V))", _HERM_PINS),
    "complex principal angles: transpose without conjugation": (
        "principal_angles_complex", "X - Y @ (Y.conj().T @ X)", "X - Y @ (Y.T @ X)", _HERM_PINS),
}


@pytest.mark.parametrize("name", sorted(SOURCE_MUTATIONS))
def test_planted_source_mistake_is_caught(monkeypatch, name):
    fname, old, new, pins = SOURCE_MUTATIONS[name]
    monkeypatch.setattr(O, fname, _source_mutant(getattr(O, fname), old, new))
    caught = False
    for pin in pins:
        try:
            pin()
        except Exception:
            caught = True
            break
    assert caught, f"no pin caught: {name}"


# ---- the warm-start network's reference

from oracle import fno_oracle as F  # noqa: E402
from tests import test_fno_oracle as TF  # noqa: E402

_FNO_PINS = [TF.test_forward_composes_the_layers_as_defined, TF.test_zero_network_outputs_the_prior_plus_output_bias,
             TF.test_spectral_layer_reproduces_low_sine_modes, TF.test_loss_is_sum_of_squared_principal_angle_sines,
             TF.test_adam_first_step_moves_each_weight_by_lr, TF.test_gradient_matches_central_differences,
             TF.test_bf16_rounding_is_the_library_conversion]

FNO_MUTATIONS = {
    "network: gelu left out of the hidden layers": (
        "forward", 'U = gelu(spectral(U, P[f"R{l}"], S) + pointwise(U, P[f"W{l}"], P[f"b{l}"]))',
        'U = spectral(U, P[f"R{l}"], S) + pointwise(U, P[f"W{l}"], P[f"b{l}"])'),
    "network: output spectral term dropped": ("forward", '+ spectral(U, P["R_out"], S) +', "+"),
    "network: prior dropped": ("forward", "return prior(cfg.N, cfg.p)[None] + spectral", "return spectral"),
    "network: sine transform transposed": ("spectral", "Uh = S @ U @ S.T", "Uh = S.T @ U @ S"),
    "network: pointwise bias dropped": ("pointwise", " + b[None, :, None, None]", ""),
    "loss: G^-1 left out": ("subspace_loss", "torch.linalg.solve(G, M)", "M"),
    "adam: no bias correction of the first moment": ("adam_step", "mh = m / (1.0 - beta1 ** t)", "mh = m"),
    "adam: second moment not squared": ("adam_step", "(1.0 - beta2) * grad * grad", "(1.0 - beta2) * grad"),
    "bfloat16: truncation instead of rounding": ("round_bf16", "bits = ((kept + up) << 16)", "bits = (kept << 16)"),
    "bfloat16: ties away from zero": ("round_bf16", "up = (rest > 0x8000) | ((rest == 0x8000) & (kept & 1 == 1))",
                                      "up = rest >= 0x8000"),
}


@pytest.mark.parametrize("name", sorted(FNO_MUTATIONS))
def test_planted_network_mistake_is_caught(monkeypatch, name):
    fname, old, new = FNO_MUTATIONS[name]
    monkeypatch.setattr(F, fname, _source_mutant(getattr(F, fname), old, new))
    caught = False
    for pin in _FNO_PINS:
        try:
            with np.errstate(all="ignore"):
                pin()
        except Exception:
            caught = True
            break
    assert caught, f"no pin caught: {name}"
