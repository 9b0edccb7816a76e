"""Pins of the RK(5,3) pseudo-time driver reference (no GPU): the harmonic iteration's
fixed point is the solution of the linearised system, whatever K and the stage
coefficients (implicit and explicit schemes reach the same dense solution); a uniform
state is steady; the mean-flow residual falls from the smooth synthetic state."""
import numpy as np
import pytest

from oracle import assemble, ordering, rk, solve
from paper_2404_01407_amd import synth


@pytest.fixture(scope="module")
def small():
    m = synth.passage_block(6, 4, 3, 36, seed=5)
    Q = synth.flow_state(m, 5)
    col = ordering.bipartite_colouring(m.n_cells, m.edges)
    return m, Q, col


def test_stage_coefficients_are_consistent():
    # the last stage has alpha = 1 (a full step); beta blends to a convex combination
    assert rk.ALPHA[-1] == 1.0 and all(0.0 < a <= 1.0 for a in rk.ALPHA)
    assert all(0.0 <= b <= 1.0 for b in rk.BETA) and rk.BETA[0] == 1.0


# explicit: P = J_ii holds half the sum of the face spectral radii, so Gamma alpha P^-1
# with sigma_CFL = 1 is a local step of CFL 2 (the five-stage scheme diverges at 4)
@pytest.mark.parametrize("scheme,sigma", [("implicit", 50.0), ("explicit", 1.0)])
def test_harmonic_fixed_point_is_the_linearised_solution(small, scheme, sigma):
    m, Q, col = small
    om = np.array([18.0])
    rng = np.random.default_rng(1)
    fh = rng.standard_normal((m.n_cells, 6)) + 1j * rng.standard_normal((m.n_cells, 6))
    J = assemble.residual_jacobian(Q, m.edges, m.area, m.bface_cell, m.bface_area)
    x_star = solve.dense_solve(J, m.volume, m.zone, om, fh)
    Qh = np.zeros_like(fh)
    hist = []
    for _ in range(400):
        Qh, r = rk.harmonic_step(m, Q, Qh, fh, om, col, sigma=sigma, scheme=scheme)
        hist.append(r)
        if r <= 1e-11 * hist[0]:
            break
    assert np.linalg.norm(Qh - x_star) <= 1e-8 * np.linalg.norm(x_star), (scheme, len(hist), hist[-1] / hist[0])
    # a flipped residual sign walks away from the solution instead
    Qw, _ = rk.harmonic_step(m, Q, np.zeros_like(fh), -fh, om, col, sigma=sigma, scheme=scheme)
    Qg, _ = rk.harmonic_step(m, Q, np.zeros_like(fh), fh, om, col, sigma=sigma, scheme=scheme)
    assert np.linalg.norm(Qg - x_star) < np.linalg.norm(Qw - x_star)


def test_uniform_state_is_steady(small):
    m, _, col = small
    q = np.array([1.0, 0.5, 0.1, -0.2, 2.7, 1e-4])
    Q = np.tile(q, (m.n_cells, 1))
    assert np.abs(rk.nonlinear_residual(m, Q)).max() <= 1e-14
    Q1, r0 = rk.mean_step(m, Q, col)
    np.testing.assert_allclose(Q1, Q, rtol=0, atol=1e-13)


def test_mean_residual_falls(small):
    m, Q, col = small
    r = []
    for _ in range(15):
        Q, rn = rk.mean_step(m, Q, col)
        r.append(rn)
    assert r[-1] < 0.5 * r[0], r
    assert np.all(np.isfinite(Q))
