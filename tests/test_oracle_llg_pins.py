"""Pins of the LLG reference (Sec. 2) against closed-form motion.

A single cubic cell has a demagnetizing field parallel to m (N = I/3), which
exerts no torque, so in a uniform external field H along z the moment moves
as the analytic solution of the LLG equation:
  azimuth  phi(t) = phi0 + g H t           (precession, g = gamma/(1+alpha^2)),
  polar    tan(theta/2) = tan(theta0/2) exp(-alpha g H t)   (damping).
Heun is second order: the error falls by ~4 when dt halves.
"""
import numpy as np

import oracle
from oracle import llg

GAMMA = 2.2128e5


def analytic(theta0, phi0, alpha, H, t):
    g = GAMMA / (1 + alpha ** 2)
    theta = 2 * np.arctan(np.tan(theta0 / 2) * np.exp(-alpha * g * H * t))
    phi = phi0 + g * H * t
    return np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])


def run_cell(alpha, H, dt, steps, theta0=1.0, phi0=0.3):
    o = oracle.Oracle((1, 1, 1), (2e-9,) * 3)
    m0 = np.array([np.sin(theta0) * np.cos(phi0), np.sin(theta0) * np.sin(phi0), np.cos(theta0)]).reshape(3, 1, 1, 1)
    m = llg.heun(lambda x: o.field(x, 8e5), m0, alpha, GAMMA, (0, 0, H), dt, steps)
    return m.reshape(3), analytic(theta0, phi0, alpha, H, dt * steps)


def test_precession_and_damping_match_closed_form_second_order():
    H = 8e4
    for alpha in (0.0, 0.1, 1.0):
        g = GAMMA / (1 + alpha ** 2)
        T = 3.0 / (g * H)  # about half a precession period
        errs = []
        for steps in (100, 200, 400):
            got, ref = run_cell(alpha, H, T / steps, steps)
            errs.append(np.abs(got - ref).max())
        assert errs[-1] < 2e-5, (alpha, errs)
        assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0, (alpha, errs)


def test_unit_length_and_torque_free_demag_of_single_cube():
    got, _ = run_cell(0.5, 0.0, 1e-13, 50)
    m0 = np.array([np.sin(1.0) * np.cos(0.3), np.sin(1.0) * np.sin(0.3), np.cos(1.0)])
    assert abs(np.linalg.norm(got) - 1) < 1e-14
    assert np.abs(got - m0).max() < 1e-14  # H_demag || m: nothing moves


def test_damped_demag_relaxation_lowers_energy():
    """alpha > 0, demag only: the stray-field energy does not increase."""
    from paper_1204_4302_amd import inputs
    shape, cell, Ms = (8, 4, 2), (2e-9, 2e-9, 2e-9), 8e5
    o = oracle.Oracle(shape, cell)
    m = inputs.random_unit(shape, 9)
    energies = []
    for _ in range(6):
        energies.append(o.energy(m, o.field(m, Ms), Ms))
        m = llg.heun(lambda x: o.field(x, Ms), m, 0.8, GAMMA, (0, 0, 0), 5e-14, 10)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(energies, energies[1:])), energies
