"""The oracle's pins are sensitive: each plausible mistake, planted into the oracle on the
CPU, makes at least one pin fail."""
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
