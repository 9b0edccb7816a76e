"""Pins of the learned-preconditioner reference (no GPU): finite differences of the
loss, positive homogeneity, relabelling equivariance, the two-hop receptive field, a
hand-worked first Adam step, the pass-through weights that make the network the
block-Jacobi correction (closed form), and the line step along a correction: exact
directions give the inverse scale, orthogonal ones nothing, the acceptance threshold
on directions of known gain, non-finite directions rejected."""
import numpy as np
import pytest

from oracle import assemble, learned, solve
from paper_2404_01407_amd import synth


@pytest.fixture(scope="module")
def small():
    m = synth.passage_block(4, 3, 3, 36, seed=21)
    Q = synth.flow_state(m, 21)
    K = assemble.assemble(m, Q)
    om = np.array([18.0])
    Ds = solve.system_diag(K, m.volume, m.zone, om)
    rng = np.random.default_rng(0)
    r = rng.standard_normal((m.n_cells, 6)) + 1j * rng.standard_normal((m.n_cells, 6))
    e = rng.standard_normal((m.n_cells, 6)) + 1j * rng.standard_normal((m.n_cells, 6))
    return m, K, Ds, r, e


def test_param_count():
    assert learned.n_params() == 60 * 64 + 88 * 64 + 128 * 64 + 128 * 64 + 64 * 12


def _loss(w, K, Ds, r, e):
    u, g, sigma = learned.features(K, Ds, r)
    return learned.loss_and_grad(w, u, g, K.rows, K.cols, r.shape[0], learned.c2r(e / sigma))


def test_gradient_finite_differences(small):
    m, K, Ds, r, e = small
    w = learned.init_weights(1)
    w[-768:] *= 10.0   # undo the small decoder init so every layer carries signal
    L, grad = _loss(w, K, Ds, r, e)
    u, g, sigma = learned.features(K, Ds, r)
    ehat = learned.c2r(e / sigma)

    def Lof(ww):
        return learned.loss_and_grad(ww, u, g, K.rows, K.cols, m.n_cells, ehat)[0]

    rng = np.random.default_rng(2)
    # directional derivative along random directions (checks the whole gradient)
    for _ in range(4):
        v = rng.standard_normal(w.size)
        h = 1e-6
        fd = (Lof(w + h * v) - Lof(w - h * v)) / (2 * h)
        assert abs(fd - grad @ v) <= 1e-6 * max(1.0, abs(fd))
    # individual weights spread over all five matrices
    offs = np.cumsum([0] + [a * b for a, b in learned.SHAPES])
    idx = np.concatenate([rng.integers(offs[k], offs[k + 1], 40) for k in range(5)])
    for i in idx:
        h = 1e-5 * max(1.0, abs(w[i]))
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (Lof(wp) - Lof(wm)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(grad).max()), i


def test_positive_homogeneity(small):
    m, K, Ds, r, e = small
    w = learned.init_weights(3)
    d1 = learned.apply(w, K, Ds, r)
    d2 = learned.apply(w, K, Ds, 7.5 * r)
    np.testing.assert_allclose(d2, 7.5 * d1, rtol=1e-12, atol=1e-14 * np.abs(d2).max())


def test_two_hop_receptive_field(small):
    m, K, Ds, r, e = small
    w = learned.init_weights(4)
    d0 = learned.apply(w, K, Ds, r)
    # perturb r at one cell, far from the boundary of the change: cells more than two
    # hops away keep their output; the scale sigma is held fixed by compensating
    c = 5
    r2 = r.copy()
    r2[c] = r[c] * np.exp(0.7j)          # same modulus: sigma unchanged
    d1 = learned.apply(w, K, Ds, r2)
    adj = [set() for _ in range(m.n_cells)]
    for a, b in m.edges:
        adj[a].add(b)
        adj[b].add(a)
    hop1 = adj[c] | {c}
    hop2 = set().union(*[adj[k] for k in hop1]) | hop1
    hop3 = set().union(*[adj[k] for k in hop2]) | hop2
    changed = {i for i in range(m.n_cells) if np.abs(d1[i] - d0[i]).max() > 1e-13}
    assert changed <= hop3          # g_ij carries z_j one more hop
    assert c in changed and len(changed & (hop2 - hop1)) > 0


def test_relabelling_equivariance(small):
    m, K, Ds, r, e = small
    w = learned.init_weights(5)
    rng = np.random.default_rng(8)
    p = rng.permutation(m.n_cells)          # old -> new
    inv = np.argsort(p)
    K2 = K.copy()
    K2.rows = p[K.rows]
    K2.cols = p[K.cols]
    K2.diag = K.diag[inv]
    d0 = learned.apply(w, K, Ds, r)
    d1 = learned.apply(w, K2, Ds[inv], r[inv])
    np.testing.assert_allclose(d1, d0[inv], rtol=1e-12, atol=1e-13 * np.abs(d0).max())


def test_adam_first_step_closed_form():
    # first step: m_hat = g, v_hat = g^2, so w1 = w0 - lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 0.0, 1e-3])
    w0 = np.array([1.0, 2.0, 3.0, 4.0])
    opt = learned.Adam(4, lr=0.01, eps=1e-8)
    w1 = opt.step(w0, g)
    np.testing.assert_allclose(w1, w0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-15)
    np.testing.assert_allclose(w1[:2], [0.99, 2.01], rtol=1e-9)


def test_block_jacobi_weights_give_the_diagonal_solve(small):
    m, K, Ds, r, e = small
    d = learned.apply(learned.block_jacobi_weights(), K, Ds, r)
    z = np.array([np.linalg.solve(Ds[i], r[i]) for i in range(m.n_cells)])      # per-cell 6x6 solves
    assert np.linalg.norm(d - z) <= 1e-13 * np.linalg.norm(z)


def _orth(rng, r):
    """A random vector orthogonal to r, scaled to ||r||."""
    q = rng.standard_normal(r.shape) + 1j * rng.standard_normal(r.shape)
    q = q - (np.vdot(r, q) / np.vdot(r, r)) * r
    return q * (np.linalg.norm(r) / np.linalg.norm(q))


def test_line_step_closed_forms(small):
    m, K, Ds, r, e = small
    A = lambda v: solve.apply(K, Ds, v)
    Ainv = lambda v: solve.dense_solve(K, m.volume, m.zone, np.array([18.0]), v)
    rng = np.random.default_rng(4)
    c = 2.0 - 3.0j
    alpha, gain = learned.line_step(A, r, c * Ainv(r))             # exact direction, scaled
    assert abs(alpha - 1.0 / c) <= 1e-10 * abs(1.0 / c) and abs(gain - 1.0) <= 1e-10
    q = _orth(rng, r)
    alpha, gain = learned.line_step(A, r, Ainv(q))                  # A d orthogonal to r
    assert alpha == 0.0 and gain <= 1e-20
    # A d = r + t q with q orthogonal to r, ||q|| = ||r||: gain 1 / (1 + t^2), alpha = gain
    for target, kept in ((2e-3, True), (0.5e-3, False)):
        t = np.sqrt(1.0 / target - 1.0)
        alpha, gain = learned.line_step(A, r, Ainv(r + t * q))
        assert abs(gain - target) <= 1e-8 * target
        assert (alpha != 0.0) == kept
        if kept:
            assert abs(alpha - target) <= 1e-8 * target
    bad = Ainv(r)
    bad[3, 2] = np.nan
    assert learned.line_step(A, r, bad)[0] == 0.0
    assert learned.line_step(A, r, np.zeros_like(r))[0] == 0.0
