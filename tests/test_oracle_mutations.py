"""Planted mistakes in the oracle must fail at least one pin.

Each case monkeypatches one plausible error into the CPU oracle (a wrong
sign, a swapped composition order, a dropped factor) and checks that the
pin tests of ``test_oracle_pins`` reject it.  Nothing here touches a GPU.
"""
import numpy as np
import pytest

import test_oracle_sgt as hpins
import test_oracle_pins as pins
from oracle import fista as F, instance as I, sgt as OH


def _rotate_wrong_sign(z, first, second, c, s, transpose=False):
    zi, zj = z[first].copy(), z[second].copy()
    sg = -1.0 if transpose else 1.0
    z[first] = c * zi + sg * s * zj        # should be c zi - s zj
    z[second] = -sg * s * zi + c * zj
    return z


def test_wrong_givens_sign_is_caught(monkeypatch):
    monkeypatch.setattr(I, "rotate", _rotate_wrong_sign)
    with pytest.raises(AssertionError):
        pins.test_givens_explicit_matrix_entries()


def test_wrong_composition_order_is_caught(monkeypatch):
    def apply_Gt_wrong(self, x):
        z = np.array(x, dtype=np.float64, copy=True)
        for st in self.G_stages:           # should run S_r^T first
            I.rotate(z, st.first, st.second, st.c, st.s, transpose=True)
        return z
    monkeypatch.setattr(I.Instance, "apply_Gt", apply_Gt_wrong)
    with pytest.raises(AssertionError):
        pins.test_operator_equals_definition_by_matrix_products(pins.SMALL[1])


def test_wrong_stage_direction_on_m_side_is_caught(monkeypatch):
    def apply_Q_wrong(self, z):
        z = np.array(z, dtype=np.float64, copy=True)
        for st in self.Q_stages:
            I.rotate(z, st.first, st.second, st.c, st.s, transpose=True)
        return z
    monkeypatch.setattr(I.Instance, "apply_Q", apply_Q_wrong)
    with pytest.raises(AssertionError):
        pins.test_operator_equals_definition_by_matrix_products(pins.SMALL[0])


def test_dropped_tau_in_noise_is_caught(monkeypatch):
    orig = I.Instance._make_solution

    def make_wrong(self, key):
        tau = self.tau
        self.tau = 1.0                     # e built without tau
        orig(self, key)
        self.tau = tau
        self.fstar = tau * np.abs(self.xstar).sum() + 0.5 * self.e @ self.e
    monkeypatch.setattr(I.Instance, "_make_solution", make_wrong)
    with pytest.raises(AssertionError):
        pins.test_planted_solution_is_optimal(pins.SMALL[0])


def test_sigma_instead_of_inverse_in_noise_is_caught(monkeypatch):
    orig_sigma = I.sigma_values
    inst_cls = I.Instance
    orig = inst_cls._make_solution

    def make_wrong(self, key):
        sig = self.sigma
        self.sigma = 1.0 / sig             # Sigma in place of Sigma^{+T}
        orig(self, key)
        self.sigma = sig
        self.b = self.matvec(self.xstar) + self.e
    monkeypatch.setattr(inst_cls, "_make_solution", make_wrong)
    with pytest.raises(AssertionError):
        pins.test_igen_noise_matches_literal_formula(pins.SMALL[1])
    assert orig_sigma is I.sigma_values


def test_wrong_momentum_is_caught(monkeypatch):
    def fista_wrong(A_mv, At_mv, b, tau, L, iters, x0=None, return_y=False):
        n = At_mv(np.zeros_like(b)).shape[0]
        x = np.zeros(n)
        y = x.copy()
        t = 1.0
        for _ in range(iters):
            x_new = F.soft_threshold(y - At_mv(A_mv(y) - b) / L, tau / L)
            t_new = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
            y = x_new + (t / t_new) * (x_new - x)      # should be (t-1)/t_new
            x, t = x_new, t_new
        return x
    monkeypatch.setattr(F, "fista", fista_wrong)
    with pytest.raises(AssertionError):
        pins.test_fista_lyapunov_nonincreasing()


def test_wrong_threshold_is_caught(monkeypatch):
    orig = F.soft_threshold
    monkeypatch.setattr(F, "soft_threshold", lambda z, thr: orig(z, 2.0 * thr))
    with pytest.raises(AssertionError):
        pins.test_fista_one_step_exact_for_orthonormal_columns()


def test_wrong_dual_sign_is_caught(monkeypatch):
    def dual_wrong(At_mv, b, tau, r):
        g_inf = float(np.abs(At_mv(r)).max())
        theta = 1.0 if g_inf <= tau else tau / g_inf
        u = theta * r
        return -0.5 * float(u @ u) + float(b @ u)        # sign of b^T u flipped
    monkeypatch.setattr(F, "dual_value", dual_wrong)
    with pytest.raises(AssertionError):
        pins.test_duality_gap_brackets_optimum()


# ---- section 8.9 class -------------------------------------------------------
def test_sgt_wrong_givens_sign_is_caught(monkeypatch):
    monkeypatch.setattr(OH, "rotate", _rotate_wrong_sign)
    with pytest.raises(AssertionError):
        hpins.test_operator_equals_definition(64, 6)


def test_sgt_swapped_sigma_law_is_caught(monkeypatch):
    orig = OH.SgtInstance.__init__

    def init_wrong(self, n, s, seed, **kw):
        kw["sigma_odd"], kw["sigma_even"] = kw.get("sigma_even", 100.0), kw.get("sigma_odd", 0.1)
        orig(self, n, s, seed, **kw)
    monkeypatch.setattr(OH.SgtInstance, "__init__", init_wrong)
    with pytest.raises(AssertionError):
        hpins.test_sampled_values_equal_whole_construction(64, 6)


def test_sgt_dropped_tau_in_noise_is_caught(monkeypatch):
    orig = OH.SgtInstance.__init__

    def init_wrong(self, n, s, seed, **kw):
        tau = kw.get("tau", 1.0)
        orig(self, n, s, seed, **kw)
        self.e[: self.n] = self.apply_Gt(self.g) / self.sigma     # tau dropped
        self.b = self.matvec(self.xstar) + self.e
        self.tau = tau
    monkeypatch.setattr(OH.SgtInstance, "__init__", init_wrong)
    with pytest.raises(AssertionError):
        hpins.test_planted_solution_is_optimal(130, 9, 0.37)


def test_sgt_swapped_support_values_are_caught(monkeypatch):
    orig = OH.SgtInstance.__init__

    def init_wrong(self, n, s, seed, **kw):
        kw["x_neg"], kw["x_pos"] = kw.get("x_pos", 0.1), kw.get("x_neg", -1.0e4)
        orig(self, n, s, seed, **kw)
    monkeypatch.setattr(OH.SgtInstance, "__init__", init_wrong)
    with pytest.raises(AssertionError):
        hpins.test_support_values_and_subgradient(130, 9)   # odd s: floor(s/2) != s - floor(s/2)


def test_pcdm_beta_without_overlap_term_is_caught(monkeypatch):
    # beta = 1 (omega - 1 dropped) for fully parallel updates: the Jacobi step
    # with L_i overshoots on coupled pairs
    orig = OH.pcdm

    def pcdm_wrong(I, tau, iters, p=1.0, x0=None, omega=2):
        return orig(I, tau, iters, p=p, x0=x0, omega=1)
    monkeypatch.setattr(OH, "pcdm", pcdm_wrong)
    with pytest.raises(AssertionError):
        hpins.test_pcdm_single_coordinate_step_is_exact_minimisation()
