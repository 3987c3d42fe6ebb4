"""Thin-film design with the adjoint gradients: an anti-reflection coating as
in the paper's TMM-Torch example (MSE of R against zero, L-BFGS-B)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_lbfgs_anti_reflection_coating_lowers_reflectance():
    from paper_2111_13667_amd import optimize
    rng = np.random.default_rng(0)
    n_layers = [2.35, 1.46] * 4
    d0 = rng.uniform(20, 150, len(n_layers))
    wl = np.linspace(500, 900, 81)
    th = np.deg2rad(np.linspace(0, 60, 7))
    d, hist, res = optimize.design(n_layers, 1.0, 1.52, wl, th, 0.0, d0, bounds=(0.0, 400.0), max_iter=60)
    assert hist[-1] < 0.2 * hist[0], (hist[0], hist[-1])
    assert min(hist) <= hist[-1] + 1e-15
    # the objective's gradient agrees with central differences at the optimum's neighbourhood
    f = optimize.reflectance_objective(n_layers, 1.0, 1.52, wl, th, 0.0)
    x = d0
    _, g = f(x)
    v = rng.normal(size=x.size)
    h = 1e-4
    fd = (f(x + h * v)[0] - f(x - h * v)[0]) / (2 * h)
    assert abs(fd - g @ v) <= 1e-6 * abs(g @ v) + 1e-14


def test_environment_reward():
    from paper_2111_13667_amd import optimize
    assert optimize.reward([0.1, 0.2], [0.0, 0.5]) == pytest.approx(-0.4)
