"""Pins of the oracle's flux, flux Jacobian and first-order residual Jacobian against
closed forms, Euler's homogeneity theorem, eigenvalues, complex-step derivatives and
discrete conservation (no GPU)."""
import numpy as np
import pytest

from oracle import assemble, flux
from paper_2404_01407_amd import synth

G = 1.4


def _state(rho, u, p, nut):
    u = np.asarray(u, float)
    E = p / (G - 1) + 0.5 * rho * u @ u
    return np.array([rho, *(rho * u), E, rho * nut])


def test_flux_closed_form_uniform_x():
    # rho = 1.2, u = (0.5, 0, 0), p = 0.8, nu~ = 1e-4, S = (1, 0, 0):
    # F = [rho u, rho u^2 + p, 0, 0, (rho E + p) u, rho nu~ u] with
    # rho E = p/(gamma-1) + rho u^2/2 = 2 + 0.15 = 2.15
    Q = _state(1.2, [0.5, 0, 0], 0.8, 1e-4)
    F = flux.flux(Q, np.array([1.0, 0, 0]))
    np.testing.assert_allclose(F, [0.6, 1.1, 0.0, 0.0, 1.475, 6e-5], rtol=1e-15, atol=1e-16)


def test_flux_at_rest_is_pressure_only():
    Q = _state(0.9, [0, 0, 0], 0.7, 1e-3)
    S = np.array([0.3, -0.2, 0.5])
    F = flux.flux(Q, S)
    np.testing.assert_allclose(F, [0, 0.7 * 0.3, -0.7 * 0.2, 0.7 * 0.5, 0, 0], atol=1e-15)


def _random_states(rng, n):
    rho = 1 + 0.1 * rng.standard_normal(n)
    u = 0.5 * rng.standard_normal((n, 3))
    p = 0.7 + 0.05 * rng.standard_normal(n)
    nut = 10 ** rng.uniform(-5, -3, n)
    return np.array([_state(rho[i], u[i], p[i], nut[i]) for i in range(n)])


def test_jacobian_homogeneity():
    # F is homogeneous of degree one in Q, so A(Q;S) Q = F(Q;S) (Euler's theorem)
    rng = np.random.default_rng(0)
    Q = _random_states(rng, 50)
    S = rng.standard_normal((50, 3))
    A = flux.flux_jacobian(Q, S)
    np.testing.assert_allclose(np.einsum("nij,nj->ni", A, Q), flux.flux(Q, S), rtol=1e-12, atol=1e-13)


def test_jacobian_complex_step():
    rng = np.random.default_rng(1)
    Q = _random_states(rng, 20)
    S = rng.standard_normal((20, 3))
    A = flux.flux_jacobian(Q, S)
    h = 1e-30
    for j in range(6):
        Qc = Q.astype(complex)
        Qc[:, j] += 1j * h
        col = flux.flux(Qc, S.astype(complex)).imag / h
        np.testing.assert_allclose(col, A[:, :, j], rtol=1e-13, atol=1e-14)


def test_jacobian_eigenvalues():
    # eigenvalues of A(Q;S): U (four times) and U +/- a|S|; spectral radius |U| + a|S|
    rng = np.random.default_rng(2)
    Q = _random_states(rng, 10)
    S = rng.standard_normal((10, 3))
    A = flux.flux_jacobian(Q, S)
    rho, u, p, H, nut = flux.primitives(Q)
    a = np.sqrt(G * p / rho)
    U = np.sum(u * S, 1)
    nS = np.linalg.norm(S, axis=1)
    for n in range(10):
        ev = np.sort(np.linalg.eigvals(A[n]).real)
        want = np.sort([U[n]] * 4 + [U[n] + a[n] * nS[n], U[n] - a[n] * nS[n]])
        np.testing.assert_allclose(ev, want, atol=1e-6)
    np.testing.assert_allclose(flux.spectral_radius(Q, S), np.abs(U) + a * nS, rtol=1e-15)


@pytest.fixture(scope="module")
def tiny():
    m = synth.passage_block(3, 2, 2, 36, seed=4)
    Q = synth.flow_state(m, 4)
    return m, Q


def test_residual_jacobian_complex_step(tiny):
    # J = dR/dQ with frozen lambda, column by column from the residual function
    m, Q = tiny
    n = m.n_cells
    J = assemble.residual_jacobian(Q, m.edges, m.area, m.bface_cell, m.bface_area)
    lam_e, lam_f, Qf = assemble.frozen_lambdas(Q, m.edges, m.area, m.bface_cell, m.bface_area)
    dense = np.zeros((6 * n, 6 * n))
    for i in range(n):
        dense[6 * i:6 * i + 6, 6 * i:6 * i + 6] = J.diag[i]
    for e in range(J.rows.shape[0]):
        dense[6 * J.rows[e]:6 * J.rows[e] + 6, 6 * J.cols[e]:6 * J.cols[e] + 6] += J.offd[e]
    h = 1e-30
    for c in range(n):
        for j in range(6):
            Qc = Q.astype(complex)
            Qc[c, j] += 1j * h
            R = assemble.residual(Qc, m.edges, m.area.astype(complex), m.bface_cell,
                                  m.bface_area.astype(complex), lam_e, lam_f, Qf.astype(complex))
            col = (R.imag / h).reshape(-1)
            np.testing.assert_allclose(col, dense[:, 6 * c + j], rtol=1e-12, atol=1e-14)


def test_discrete_conservation(tiny):
    # interior faces conserve: the block-column sum of J over all rows equals the
    # boundary-face contributions of that cell only
    m, Q = tiny
    J = assemble.residual_jacobian(Q, m.edges, m.area, m.bface_cell, m.bface_area)
    colsum = J.diag.copy()
    np.add.at(colsum, J.cols, J.offd)
    lam_e, lam_f, Qf = assemble.frozen_lambdas(Q, m.edges, m.area, m.bface_cell, m.bface_area)
    want = np.zeros_like(colsum)
    Af = flux.flux_jacobian(Q[m.bface_cell], m.bface_area)
    np.add.at(want, m.bface_cell, 0.5 * Af + 0.5 * lam_f[:, None, None] * np.eye(6))
    np.testing.assert_allclose(colsum, want, rtol=1e-12, atol=1e-15)


def test_closed_cell_diagonal_is_scalar():
    # sum of outward area vectors of a closed cell vanishes and A is linear in S, so
    # J_ii = (1/2) sum_faces lambda_f I exactly
    m = synth.passage_block(5, 4, 3, 36, seed=7)
    Q = synth.flow_state(m, 7)
    J = assemble.residual_jacobian(Q, m.edges, m.area, m.bface_cell, m.bface_area)
    lam_e, lam_f, _ = assemble.frozen_lambdas(Q, m.edges, m.area, m.bface_cell, m.bface_area)
    s = np.zeros(m.n_cells)
    np.add.at(s, m.edges[:, 0], lam_e)
    np.add.at(s, m.edges[:, 1], lam_e)
    np.add.at(s, m.bface_cell, lam_f)
    want = 0.5 * s[:, None, None] * np.eye(6)
    scale = np.abs(J.diag).max()
    assert np.abs(J.diag - want).max() <= 1e-12 * scale


def test_preconditioner_matrix_forms(tiny):
    m, Q = tiny
    J = assemble.residual_jacobian(Q, m.edges, m.area, m.bface_cell, m.bface_area)
    K = assemble.preconditioner_matrix(J, eps=0.6, sigma=50.0)
    np.testing.assert_array_equal(K.offd, J.offd)
    np.testing.assert_allclose(K.diag, J.diag * (1 + 1 / 30.0), rtol=1e-15)
    Ke = assemble.preconditioner_matrix(J, scheme="explicit")
    assert not Ke.offd.any()
    np.testing.assert_array_equal(Ke.diag, J.diag)
