"""Pins of the partition-dropped preconditioner matrix (no GPU): its dense form is the full
one with every block between two partitions struck out and nothing else changed; one
partition leaves K unchanged; one cell per partition leaves the block diagonal, which
the Richardson iteration solves exactly in one sweep; the solve splits into independent
per-partition solves; and the RK iteration converges more slowly as the partitions
shrink (the paper's degradation rule, in kind).  Also the bisection partition generator.
Partition-local ILU(0) in the natural order, as the oracle of the GPU's "pilu" kind
(DILU with every cell its own class, in id order, on the dropped matrix): on a hex mesh
(no triangles in the cell graph) it is the textbook block ILU(0) in id order, and its
preconditioner splits into each partition's own ILU(0) of its own block of K."""
import numpy as np
import pytest

from oracle import assemble, ordering, rk, solve
from paper_2404_01407_amd import synth


@pytest.fixture(scope="module")
def small():
    m = synth.passage_block(8, 4, 4, 36, seed=8)
    Q = synth.flow_state(m, 8)
    K = assemble.assemble(m, Q)
    col = ordering.bipartite_colouring(m.n_cells, m.edges)
    return m, Q, K, col


def _b(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, 6)) + 1j * rng.standard_normal((n, 6))


@pytest.mark.parametrize("size", [1, 3, 16, 40, 128])
def test_rcb_partition_sizes(small, size):
    m = small[0]
    part = synth.rcb_partition(m, size)
    counts = np.bincount(part)
    assert counts.sum() == m.n_cells and counts.max() <= size
    assert counts.min() >= size // 2 or size >= m.n_cells            # halving keeps parts balanced
    assert np.array_equal(part, synth.rcb_partition(m, size))        # deterministic


def test_dense_is_the_full_dense_struck_out(small):
    m, Q, K, col = small
    part = synth.rcb_partition(m, 16)
    om = np.array([18.0])
    A = solve.dense(K, m.volume, m.zone, om)
    Ad = solve.dense(solve.partition_dropped(K, part), m.volume, m.zone, om)
    same = np.equal.outer(np.repeat(part, 6), np.repeat(part, 6))
    assert np.array_equal(Ad[same], A[same])
    assert not np.any(Ad[~same])
    assert np.any(A[~same])                                          # something was dropped


def test_one_partition_is_k(small):
    m, Q, K, col = small
    Kd = solve.partition_dropped(K, np.zeros(m.n_cells, np.int32))
    assert np.array_equal(Kd.offd, K.offd) and np.array_equal(Kd.diag, K.diag)


def test_single_cells_leave_the_block_diagonal(small):
    m, Q, K, col = small
    Kd = solve.partition_dropped(K, np.arange(m.n_cells))
    om = np.array([27.0])
    b = _b(m.n_cells, 1)
    x, info = solve.richardson(Kd, m.volume, m.zone, om, b, col, "DILU", rtol=1e-13, max_sweeps=3)
    xd = np.linalg.solve(solve.system_diag(K, m.volume, m.zone, om), b[..., None])[..., 0]
    assert info.sweeps == 1
    assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd)


def test_solve_splits_into_partitions(small):
    m, Q, K, col = small
    part = synth.rcb_partition(m, 40)
    om = np.array([18.0])
    b = _b(m.n_cells, 2)
    x = solve.dense_solve(solve.partition_dropped(K, part), m.volume, m.zone, om, b)
    A = solve.dense(K, m.volume, m.zone, om)
    for p in np.unique(part):
        cells = np.nonzero(part == p)[0]
        idx = (6 * cells[:, None] + np.arange(6)).ravel()
        xp = np.linalg.solve(A[np.ix_(idx, idx)], b[cells].reshape(-1))   # the partition's own block of K
        np.testing.assert_allclose(x[cells].reshape(-1), xp, rtol=0, atol=1e-10 * np.abs(xp).max())


def test_rk_converges_slower_with_smaller_partitions(small):
    m, Q, K, col = small
    om = np.array([18.0])
    fh = _b(m.n_cells, 3)
    steps = []
    # CFL 50: 7, 14, 30, 102 steps for parts of 128, 64, 32, 16 cells; parts of 8 cells or
    # fewer diverge (towards single cells the stage update becomes a local explicit step
    # of CFL ~ 2 sigma / (1 + eps sigma) ~ 3, beyond the five-stage scheme's limit here)
    for size in (m.n_cells, 64, 32, 16):
        part = synth.rcb_partition(m, size)
        Qh = np.zeros_like(fh)
        hist = []
        for n in range(200):
            Qh, r = rk.harmonic_step(m, Q, Qh, fh, om, col, part=part)
            hist.append(r)
            if r <= 1e-6 * hist[0]:
                break
        steps.append(n + 1)
        J = assemble.residual_jacobian(Q, m.edges, m.area, m.bface_cell, m.bface_area)
        x_star = solve.dense_solve(J, m.volume, m.zone, om, fh)      # the same fixed point whatever the split
        assert np.linalg.norm(Qh - x_star) <= 1e-4 * np.linalg.norm(x_star), (size, n, hist[-1] / hist[0])
    assert steps[0] < steps[1] < steps[2] < steps[3], steps


def _sub_matrix(K, cells):
    """The partition's own block of K as a BlockMatrix on its cells (renumbered 0..)."""
    loc = -np.ones(K.n, np.int64)
    loc[cells] = np.arange(cells.size)
    keep = np.nonzero((loc[K.rows] >= 0) & (loc[K.cols] >= 0))[0]
    return assemble.BlockMatrix(cells.size, K.diag[cells].copy(), loc[K.rows[keep]], loc[K.cols[keep]],
                                K.offd[keep].copy())


def test_natural_dilu_is_textbook_ilu0_per_partition(small):
    m, Q, K, col = small
    part = synth.rcb_partition(m, 24)
    Kd = solve.partition_dropped(K, part)
    om = np.array([18.0])
    r = _b(m.n_cells, 5)
    natural = np.arange(m.n_cells)
    f_dilu = solve.factor(Kd, m.volume, m.zone, om, natural, "DILU")
    z = solve.precondition(Kd, f_dilu, r)
    # the textbook IKJ ILU(0) in id order (one colour class: the order is the ids')
    f_ilu = solve.factor(Kd, m.volume, m.zone, om, np.zeros(m.n_cells, np.int64), "ILU0")
    z_ilu = solve.precondition(Kd, f_ilu, r)
    np.testing.assert_allclose(z, z_ilu, rtol=0, atol=1e-12 * np.abs(z).max())
    # each partition alone: its block of the undropped K, its own ILU(0) in id order
    for p in np.unique(part):
        cells = np.nonzero(part == p)[0]                               # ascending: id order kept
        Kp = _sub_matrix(K, cells)
        fp = solve.factor(Kp, m.volume[cells], m.zone[cells], om, np.zeros(cells.size, np.int64), "ILU0")
        zp = solve.precondition(Kp, fp, r[cells])
        np.testing.assert_allclose(z[cells], zp, rtol=0, atol=1e-12 * np.abs(zp).max())


def test_natural_order_differs_from_the_colouring(small):
    """The natural order is a different preconditioner from the colour ordering's (a
    mistake that handed the colouring to the natural-order kind would show here)."""
    m, Q, K, col = small
    part = synth.rcb_partition(m, 40)
    Kd = solve.partition_dropped(K, part)
    om = np.array([18.0])
    r = _b(m.n_cells, 6)
    zn = solve.precondition(Kd, solve.factor(Kd, m.volume, m.zone, om, np.arange(m.n_cells), "DILU"), r)
    zc = solve.precondition(Kd, solve.factor(Kd, m.volume, m.zone, om, col, "DILU"), r)
    assert np.linalg.norm(zn - zc) > 1e-3 * np.linalg.norm(zc)
