"""Planted mistakes in the oracle (on the CPU): each plausible mistake in a
piece of the oracle makes at least one of that piece's pins fail. The
mistakes are planted by replacing one oracle function for the duration of a
test (pytest's monkeypatch); the pins are the tests of test_oracle_*.py,
called as plain functions."""
import math

import numpy as np
import pytest

import test_oracle_projector as tproj
import test_oracle_spdhg as tspd
import test_oracle_subsets as tsub
import test_oracle_warp as twarp
from oracle import projector, spdhg, subsets, warp


def _fails(pin, *args):
    with pytest.raises(AssertionError):
        pin(*args)


# --- ray transform (Section II-A's A; Joseph discretisation) -----------------

def test_dropping_the_ray_length_fails_the_disc(monkeypatch):
    good = projector._crossings

    def no_ds(n, n_det, k, n_angles):
        cf, ds, rows = good(n, n_det, k, n_angles)
        return cf, 1.0, rows

    monkeypatch.setattr(projector, "_crossings", no_ds)
    _fails(tproj.test_off_centre_disc_matches_closed_form)


def test_swapped_interpolation_weights_fail_the_axis_cases(monkeypatch):
    good = projector._crossings

    def swapped(n, n_det, k, n_angles):
        # the fraction measured from the other tap: (1 - f) on floor + 1
        cf, ds, rows = good(n, n_det, k, n_angles)
        c0 = np.floor(cf)
        return c0 + (1.0 - (cf - c0)), ds, rows

    monkeypatch.setattr(projector, "_crossings", swapped)
    _fails(tproj.test_theta0_is_column_sums, 16, 12, 24)


def test_mirrored_detector_fails_the_disc(monkeypatch):
    good = projector._crossings

    def mirrored(n, n_det, k, n_angles):
        cf, ds, rows = good(n, n_det, k, n_angles)
        return cf[:, ::-1], ds, rows

    monkeypatch.setattr(projector, "_crossings", mirrored)
    _fails(tproj.test_off_centre_disc_matches_closed_form)


# --- warp D_i (Section II-A) ----------------------------------------------------

def test_rotation_sign_fails_the_quarter_turn(monkeypatch):
    good = warp.rigid_positions
    monkeypatch.setattr(warp, "rigid_positions", lambda n, phi, tx, ty: good(n, -phi, tx, ty))
    _fails(twarp.test_quarter_turn_is_rot90)


def test_transposed_warp_with_swapped_axes_fails_the_transpose(monkeypatch):
    good = warp.warp_adjoint
    monkeypatch.setattr(warp, "warp_adjoint", lambda b, px, py: good(b, py, px))
    _fails(twarp.test_adjoint_is_exact_transpose, "rigid")


# --- Algorithm 1 -----------------------------------------------------------------

def _iterate_with(zbar_rule=None, step_i_uses_z=False):
    """Algorithm 1 with one of the printed lines taken literally."""
    def it(ops, state, d, alpha, sigma, tau, theta, p, S):
        N = ops.n_gates
        v = state.z if step_i_uses_z else state.zbar
        x = spdhg.prox_tau_g(state.x - tau * v, tau, alpha)
        y = list(state.y)
        dz = np.zeros_like(state.z)
        dzbar = np.zeros_like(state.z)
        for i in S:
            yi = spdhg.prox_sigma_fstar(state.y[i] + sigma[i] * ops.A(i, x), sigma[i], d[i], N)
            delta = ops.At(i, yi - state.y[i])
            dz += delta
            dzbar += (theta / p[i]) * delta
            y[i] = yi
        z = state.z + dz
        if zbar_rule == "printed":   # z-bar^{k+1} = z-bar^k + sum (1 + theta/p) delta
            return spdhg.State(x, y, z, state.zbar + dz + dzbar)
        return spdhg.State(x, y, z, z + dzbar)
    return it


def test_printed_zbar_recursion_fails_the_rates(monkeypatch):
    monkeypatch.setattr(spdhg, "iterate", _iterate_with(zbar_rule="printed"))
    _fails(tspd.test_observed_rates_in_paper_regime, 4, "rigid")


def test_printed_step_one_fails_the_rates(monkeypatch):
    monkeypatch.setattr(spdhg, "iterate", _iterate_with(step_i_uses_z=True))
    _fails(tspd.test_observed_rates_in_paper_regime, 4, "rigid")


def test_doubled_tau_fails_the_contraction(monkeypatch):
    good = spdhg.step_sizes_spdhg

    def wrong(norms, alpha, N):
        sigma, tau, theta, rho = good(norms, alpha, N)
        return sigma, 2.0 * tau, theta, rho

    monkeypatch.setattr(spdhg, "step_sizes_spdhg", wrong)
    _fails(tspd.test_spdhg_second_moment_within_theorem, 3, 0.05, 1)


def test_prox_without_the_gate_count_fails_optimality(monkeypatch):
    monkeypatch.setattr(spdhg, "prox_sigma_fstar", lambda v, sigma, d, n: (v - sigma * d) / (1.0 + sigma / 2.0))
    _fails(tspd.test_prox_optimality)


# --- gates x angle subsets (Conclusions) -----------------------------------------

def test_unmasked_block_adjoint_fails_the_partition(monkeypatch):
    monkeypatch.setattr(subsets.BlockOperators, "At", lambda self, b, y: self.ops.At(self.split(b)[0], y))
    _fails(tsub.test_blocks_partition_each_gate_operator, "paired")


def test_block_zbar_without_extrapolation_fails_the_rates(monkeypatch):
    # z-bar = z: the (theta / p_b) A_b^* dy term dropped
    good = subsets.iterate

    def wrong(bops, state, d, alpha, sigma, tau, theta, p, S):
        st = good(bops, state, d, alpha, sigma, tau, theta, p, S)
        return subsets.spdhg.State(st.x, st.y, st.z, st.z.copy())

    monkeypatch.setattr(subsets, "iterate", wrong)
    _fails(tsub.test_observed_rate_in_paper_regime, "paired")


def test_rate_formula_with_wrong_exponent_fails_closed_forms(monkeypatch):
    monkeypatch.setattr(spdhg, "rate", lambda kappa, n: (1.0 - 2.0 / (n * (1.0 + math.sqrt(1.0 + kappa)))) ** (n + 1))
    _fails(tspd.test_rate_closed_forms_and_paper_claim)
