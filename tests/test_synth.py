"""Synthetic workload generator: counts, closure, volumes, determinism, graph shape."""
import numpy as np
import pytest

from oracle import ordering
from paper_2404_01407_amd import synth


def _closure(m):
    acc = np.zeros((m.n_cells, 3))
    np.add.at(acc, m.edges[:, 0], m.area)
    np.add.at(acc, m.edges[:, 1], -m.area)
    np.add.at(acc, m.bface_cell, m.bface_area)
    return np.abs(acc).max() / np.abs(m.area).max()


def test_counts_small():
    m = synth.passage_block(16, 8, 4, 36, seed=1)
    assert (m.n_cells, m.n_edges, m.n_bfaces) == (512, 1312, 448)
    assert m.volume.min() > 0
    assert _closure(m) < 1e-12
    assert ordering.bipartite_colouring(m.n_cells, m.edges) is not None
    assert not ordering.has_triangle(m.n_cells, m.edges)


@pytest.mark.slow
def test_counts_200k():
    m = synth.passage_block(80, 50, 50, 36, seed=2)
    assert (m.n_cells, m.n_edges, m.n_bfaces) == (200_000, 589_500, 21_000)
    assert m.volume.min() > 0


def test_deterministic_and_permuted():
    a = synth.passage_block(6, 5, 4, 36, seed=3)
    b = synth.passage_block(6, 5, 4, 36, seed=3)
    np.testing.assert_array_equal(a.edges, b.edges)
    np.testing.assert_array_equal(synth.flow_state(a, 3), synth.flow_state(b, 3))
    c = synth.passage_block(6, 5, 4, 36, seed=4)
    assert not np.array_equal(a.edges, c.edges)
    # orientation: area vector points from a to b
    d = a.centroid[a.edges[:, 1]] - a.centroid[a.edges[:, 0]]
    assert np.all(np.sum(d * a.area, 1) > 0)


def test_state_ranges():
    m = synth.passage_block(10, 8, 6, 36, seed=2)
    Q = synth.flow_state(m, 2)
    rho = Q[:, 0]
    u = Q[:, 1:4] / rho[:, None]
    p = 0.4 * (Q[:, 4] - 0.5 * rho * np.sum(u * u, 1))
    a = np.sqrt(1.4 * p / rho)
    mach = np.linalg.norm(u, axis=1) / a
    assert 0.95 - 1e-12 <= rho.min() and rho.max() <= 1.05 + 1e-12
    assert 0.29 <= mach.min() and mach.max() <= 0.61
    nut = Q[:, 5] / rho
    assert 1e-5 * 0.999 <= nut.min() and nut.max() <= 1e-3 * 1.001


def test_multi_row_has_triangles_and_zones():
    m = synth.multi_row(4, 6, 3, n_blades=(36, 60, 48), seed=5)
    assert m.n_zones == 3 and set(np.unique(m.zone)) == {0, 1, 2}
    assert ordering.has_triangle(m.n_cells, m.edges)
    assert ordering.bipartite_colouring(m.n_cells, m.edges) is None
    assert m.volume.min() > 0


def test_rhs_and_omegas():
    b0 = synth.rhs(100, 0, real=True)
    assert np.all(b0.imag == 0)
    np.testing.assert_array_equal(synth.rhs(100, 3), synth.rhs(100, 3))
    om = synth.omegas_single_zone(3)
    np.testing.assert_array_equal(om[:, 0], [0, 18, 36, 54])
    insts = synth.batch_instances(64, 8.0e6, seed=3)
    n = sum(i["shape"][0] * i["shape"][1] * i["shape"][2] for i in insts)
    assert len(insts) == 64 and 6.0e6 < n < 10.0e6
