"""Pins of the frozen-turbulence systems (no GPU): the 5x5 sub-system's solution solves
the first five equations of the full 6x6 system with the turbulence unknown at zero;
when the turbulence variable is decoupled the frozen solve is the full solve's first
five components, iterate by iterate; the frozen system's dense matrix is the full one
with the sixth unknown's rows and columns struck out; the RK driver's frozen fixed point
is the 5x5 linearised solution."""
import numpy as np
import pytest

from oracle import assemble, ordering, rk, solve
from paper_2404_01407_amd import synth


@pytest.fixture(scope="module")
def small():
    m = synth.passage_block(6, 4, 3, 36, seed=4)
    Q = synth.flow_state(m, 4)
    K = assemble.assemble(m, Q)
    col = ordering.bipartite_colouring(m.n_cells, m.edges)
    return m, Q, K, col


def _rhs(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, 6)) + 1j * rng.standard_normal((n, 6))


def test_frozen_solution_solves_first_five_equations(small):
    m, Q, K, col = small
    om = np.array([18.0])
    b = _rhs(m.n_cells, 1)
    x, info = solve.richardson_frozen(K, m.volume, m.zone, om, b, col, "DILU", rtol=1e-13, max_sweeps=4000)
    assert info.status == solve.OK
    assert np.all(x[:, 5] == 0.0)
    # the full 6x6 operator (its own code path, shift on all six) applied to x
    r = b - solve.apply(K, solve.system_diag(K, m.volume, m.zone, om), x)
    assert np.linalg.norm(r[:, :5]) <= 1e-11 * np.linalg.norm(b[:, :5])
    # the sixth equation is not satisfied in general (the frozen unknown is not solved for)
    assert np.linalg.norm(r[:, 5]) > 1e-3 * np.linalg.norm(b[:, 5])


def test_frozen_dense_is_the_full_dense_struck_out(small):
    m, Q, K, col = small
    om = np.array([27.0])
    A6 = solve.dense(K, m.volume, m.zone, om)
    keep = np.ones(6 * m.n_cells, bool)
    keep[5::6] = False
    A5 = solve.dense(solve.frozen_turbulence(K), m.volume, m.zone, om)
    assert np.array_equal(A5, A6[np.ix_(keep, keep)])


@pytest.mark.parametrize("kind", ["DILU", "SGS", "JACOBI"])
def test_decoupled_turbulence_frozen_equals_full(small, kind):
    """With the turbulence row and column of every block zero except the diagonal entry,
    the 6x6 iteration never mixes the sixth unknown into the others (DILU, SGS and
    Jacobi keep block-diagonal structure inside each block), so its first five components
    are the frozen iteration's, sweep by sweep."""
    m, Q, K, col = small
    Kd = K.copy()
    Kd.offd[:, 5, :] = 0.0
    Kd.offd[:, :, 5] = 0.0
    d55 = Kd.diag[:, 5, 5].copy()
    Kd.diag[:, 5, :] = 0.0
    Kd.diag[:, :, 5] = 0.0
    Kd.diag[:, 5, 5] = d55
    om = np.array([18.0])
    b = _rhs(m.n_cells, 2)
    it6, it5 = [], []
    solve.richardson(Kd, m.volume, m.zone, om, b, col, kind, rtol=0.0, max_sweeps=6, iterates=it6)
    # the frozen solve sees only the leading 5x5 blocks, whatever the sixth row holds
    solve.richardson_frozen(K, m.volume, m.zone, om, b, col, kind, rtol=0.0, max_sweeps=6, iterates=it5)
    assert len(it5) == len(it6) == 7
    for a, c in zip(it6, it5):
        np.testing.assert_allclose(a[:, :5], c, rtol=0, atol=1e-12 * np.abs(a).max())


def test_frozen_rk_fixed_point_is_the_5x5_linearised_solution(small):
    m, Q, K, col = small
    om = np.array([18.0])
    fh = _rhs(m.n_cells, 3)
    J = assemble.residual_jacobian(Q, m.edges, m.area, m.bface_cell, m.bface_area)
    x5 = solve.dense_solve(solve.frozen_turbulence(J), m.volume, m.zone, om, fh[:, :5])
    Qh = _rhs(m.n_cells, 4)                      # a non-zero sixth component is reset to 0
    hist = []
    for _ in range(300):
        Qh, r = rk.harmonic_step(m, Q, Qh, fh, om, col, frozen=True)
        hist.append(r)
        if r <= 1e-11 * hist[0]:
            break
    assert np.all(Qh[:, 5] == 0.0)
    assert np.linalg.norm(Qh[:, :5] - x5) <= 1e-8 * np.linalg.norm(x5), (len(hist), hist[-1] / hist[0])
