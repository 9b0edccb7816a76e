"""Pins of the phase-lagged periodic couplings (no GPU): a single passage with
inter-blade phase angle sigma reproduces one passage of a full wheel of identical
passages driven by a travelling wave (nodal diameter), and the phase obeys the
symmetries it must."""
import numpy as np
import pytest

from oracle import assemble, ordering, solve
from paper_2404_01407_amd import synth

NB = 36


def _setup(n_passages, permute=True, ny=4):
    m = synth.cascade_block(5, ny, 3, NB, seed=7, n_passages=n_passages, permute=permute)
    Q = synth.flow_state(m, 7)
    K = assemble.assemble(m, Q)
    return m, K


def _struct_index(m):
    """user id of structured cell (i, j, k)."""
    nx, nyt, nz = m.meta["shape"]
    return m.meta["struct_to_user"].reshape(nx, nyt, nz)


@pytest.mark.parametrize("nd", [1, 2])
def test_single_passage_matches_full_wheel(nd):
    n_p = 3
    sigma = 2.0 * np.pi * nd / n_p              # nodal diameter nd of a 3-passage wheel
    m1, K1 = _setup(1)
    m3, K3 = _setup(n_p)
    om = np.array([18.0])
    rng = np.random.default_rng(3)
    b1 = rng.standard_normal((m1.n_cells, 6)) + 1j * rng.standard_normal((m1.n_cells, 6))
    s1 = _struct_index(m1)                      # [nx, ny, nz]
    s3 = _struct_index(m3)                      # [nx, 3 ny, nz]
    ny = s1.shape[1]
    b3 = np.zeros((m3.n_cells, 6), complex)
    for p in range(n_p):
        b3[s3[:, p * ny:(p + 1) * ny, :].ravel()] = b1[s1.ravel()] * np.exp(1j * p * sigma)
    # the wheel closes on itself: its periodic edges carry n_p sigma = 2 pi nd, phase 1
    K3p = solve.phase_lagged(K3, m3.edge_phase, n_p * sigma)
    x3 = solve.dense_solve(K3p, m3.volume, m3.zone, om, b3)
    x1 = solve.dense_solve(solve.phase_lagged(K1, m1.edge_phase, sigma), m1.volume, m1.zone, om, b1)
    for p in range(n_p):
        xp = x3[s3[:, p * ny:(p + 1) * ny, :].ravel()]
        np.testing.assert_allclose(xp, x1[s1.ravel()] * np.exp(1j * p * sigma), rtol=0,
                                   atol=1e-10 * np.abs(x1).max())
    # a wrong sign of the phase breaks the equivalence
    xw = solve.dense_solve(solve.phase_lagged(K1, m1.edge_phase, -sigma), m1.volume, m1.zone, om, b1)
    assert np.abs(xw - x1).max() > 1e-3 * np.abs(x1).max()


def test_zero_and_full_turn_phase():
    m, K = _setup(1)
    K0 = solve.phase_lagged(K, m.edge_phase, 0.0)
    assert np.array_equal(K0.offd, K.offd.astype(complex))
    K2 = solve.phase_lagged(K, m.edge_phase, 2.0 * np.pi)
    np.testing.assert_allclose(K2.offd, K.offd, rtol=0, atol=1e-15 * np.abs(K.offd).max())
    Ka = solve.phase_lagged(K, m.edge_phase, 0.7)
    Kb = solve.phase_lagged(K, m.edge_phase, 0.7 + 2.0 * np.pi)
    np.testing.assert_allclose(Ka.offd, Kb.offd, rtol=0, atol=1e-14 * np.abs(K.offd).max())


def test_conjugate_symmetry_with_phase():
    # K real: solve(-omega, -sigma, conj b) = conj(solve(omega, sigma, b))
    m, K = _setup(1)
    rng = np.random.default_rng(4)
    b = rng.standard_normal((m.n_cells, 6)) + 1j * rng.standard_normal((m.n_cells, 6))
    om = np.array([36.0])
    col = ordering.bipartite_colouring(m.n_cells, m.edges)
    xp, _ = solve.richardson(solve.phase_lagged(K, m.edge_phase, 1.1), m.volume, m.zone, om, b, col, "DILU",
                             rtol=0.0, max_sweeps=12)
    xm, _ = solve.richardson(solve.phase_lagged(K, m.edge_phase, -1.1), m.volume, m.zone, -om, np.conj(b), col,
                             "DILU", rtol=0.0, max_sweeps=12)
    np.testing.assert_allclose(xm, np.conj(xp), rtol=0, atol=1e-12 * np.abs(xp).max())


def test_dilu_diagonal_is_phase_free():
    # the DILU correction K_ik Dt_k^-1 K_ki pairs a coupling with its transpose, whose
    # phases are conjugate, so Dt does not depend on sigma
    m, K = _setup(1, ny=5)                       # odd pitch count: not bipartite
    col = ordering.greedy_colouring(m.n_cells, m.edges)
    Ds = solve.system_diag(K, m.volume, m.zone, np.array([18.0]))
    Dt0, _ = solve.dilu_diagonal(K, Ds, col)
    Dt1, _ = solve.dilu_diagonal(solve.phase_lagged(K, m.edge_phase, 2.3), Ds, col)
    np.testing.assert_allclose(Dt1, Dt0, rtol=0, atol=1e-12 * np.abs(Dt0).max())


def test_phased_iteration_converges_to_dense():
    m, K = _setup(1, ny=5)
    col = ordering.greedy_colouring(m.n_cells, m.edges)
    Kp = solve.phase_lagged(K, m.edge_phase, 0.9)
    om = np.array([18.0])
    b = synth.rhs(m.n_cells, 2)
    x, info = solve.richardson(Kp, m.volume, m.zone, om, b, col, "DILU", rtol=1e-12, max_sweeps=3000)
    xd = solve.dense_solve(Kp, m.volume, m.zone, om, b)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)


def test_cascade_geometry_closes():
    for n_p in (1, 3):
        m = synth.cascade_block(6, 5, 4, NB, seed=3, n_passages=n_p)
        acc = np.zeros((m.n_cells, 3))
        np.add.at(acc, m.edges[:, 0], m.area)
        np.add.at(acc, m.edges[:, 1], -m.area)
        np.add.at(acc, m.bface_cell, m.bface_area)
        assert np.abs(acc).max() <= 1e-15
        assert int(np.count_nonzero(m.edge_phase)) == 6 * 4
        assert m.volume.min() > 0
