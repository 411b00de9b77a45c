"""Host logic of the inversion drivers on a closed-form objective (no GPU):
a convex quadratic J = 1/2 (v - v*)^T A (v - v*) with diagonal A."""
import numpy as np
import pytest

from paper_1406_1864_amd.inversion import lbfgs, line_search, prcg


class Quadratic:
    def __init__(self, n=(12, 20), seed=0, precond=True):
        rng = np.random.default_rng(seed)
        self.a = rng.uniform(1.0, 50.0, n)            # condition number ~50
        self.vs = 2500.0 + 300.0 * rng.standard_normal(n)
        self.precond = precond
        self.evals = 0

    def value(self, v):
        self.evals += 1
        r = v - self.vs
        return 0.5 * float(np.sum(self.a * r * r))

    def value_grad(self, v):
        self.evals += 1
        r = v - self.vs
        minv = 1.0 / self.a if self.precond else np.ones_like(self.a)
        return 0.5 * float(np.sum(self.a * r * r)), self.a * r, minv


def test_line_search_finds_the_minimiser_of_a_quadratic():
    q = Quadratic()
    v = np.full(q.a.shape, 2500.0)
    J0, g, _ = q.value_grad(v)
    d = -g
    alpha, J, vn = line_search(q, v, J0, g, d, 1000.0, 0.0, 1e9)   # trial within 10x of the minimiser
    exact = float(np.sum(g * g)) / float(np.sum(q.a * g * g))      # argmin along -g
    assert alpha == pytest.approx(exact, rel=1e-9)
    assert J < J0


def test_line_search_refuses_an_ascent_direction():
    q = Quadratic()
    v = np.full(q.a.shape, 2500.0)
    J0, g, _ = q.value_grad(v)
    alpha, J, vn = line_search(q, v, J0, g, g, 50.0, 0.0, 1e9)
    assert alpha == 0.0 and J == J0 and vn is v


def test_exact_diagonal_scaling_solves_in_one_step():
    """With minv = A^-1 the scaled gradient is the Newton step (the trial
    step is large enough for the quadratic fit to reach it)."""
    q = Quadratic(precond=True)
    v, hist = prcg(q, np.full(q.a.shape, 2500.0), 2, step0=1000.0, vmin=0.0, vmax=1e9)
    assert hist[1]["J"] <= 1e-18 * hist[0]["J"] + 1e-20
    assert np.allclose(v, q.vs, rtol=0, atol=1e-6)


@pytest.mark.parametrize("driver", [prcg, lbfgs])
def test_drivers_converge_without_scaling(driver):
    q = Quadratic(precond=False)
    v0 = np.full(q.a.shape, 2500.0)
    v, hist = driver(q, v0, 60, vmin=0.0, vmax=1e9)
    Js = [h["J"] for h in hist]
    assert all(b <= a for a, b in zip(Js, Js[1:]))                 # monotone
    assert Js[-1] < 1e-6 * Js[0]


def test_bounds_are_respected():
    q = Quadratic()
    q.vs[:] = 5000.0                                                # optimum above the bound
    v, _ = prcg(q, np.full(q.a.shape, 2500.0), 10, vmin=1400.0, vmax=4600.0)
    assert np.all(v <= 4600.0) and np.all(v >= 1400.0)
