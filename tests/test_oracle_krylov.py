"""Pins of the FGMRES reference (no GPU): the least-squares residual after k iterations
is the minimum over the preconditioned Krylov space built by brute force from its power
basis; full GMRES on a tiny mesh reaches the dense solution; one iteration suffices when
the preconditioner is the exact inverse; the residual history never rises within a
cycle and ends at the true residual; restarted runs converge to the dense solution.
Learned kind: an exact network converges in one iteration, a zero network is the DILU
method step for step, and the nonlinear preconditioner of a random network still reaches
the dense solution (flexible GMRES).  The controller stops evaluating the network after
exactly three rejected steps in a row, and a kept step ends a run of rejections."""
import numpy as np
import pytest

from oracle import assemble, krylov, learned, ordering, solve
from paper_2404_01407_amd import synth


def _setup(shape=(6, 4, 3), seed=6):
    m = synth.passage_block(*shape, 36, seed=seed)
    Q = synth.flow_state(m, seed)
    K = assemble.assemble(m, Q)
    col = ordering.bipartite_colouring(m.n_cells, m.edges)
    return m, K, col


def _b(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, 6)) + 1j * rng.standard_normal((n, 6))


@pytest.mark.parametrize("kind", ["DILU", "JACOBI"])
def test_residual_is_the_krylov_minimum(kind):
    m, K, col = _setup()
    om = np.array([18.0])
    b = _b(m.n_cells, 1)
    kmax = 6
    _, info = krylov.fgmres(K, m.volume, m.zone, om, b, col, kind, restart=kmax, rtol=0.0, max_iters=kmax)
    Ds = solve.system_diag(K, m.volume, m.zone, om)
    f = solve.factor(K, m.volume, m.zone, om, col, kind)

    def AM(v):                                   # A M^-1 v, M^-1 one preconditioner application
        return solve.apply(K, Ds, solve.precondition(K, f, v))

    r0 = b.reshape(-1)
    Bs = [r0]
    for _ in range(kmax - 1):
        Bs.append(AM(Bs[-1].reshape(-1, 6)).reshape(-1))
    for k in range(1, kmax + 1):
        Qb, _ = np.linalg.qr(np.stack(Bs[:k], axis=1))       # orthonormal basis of K_k(A M^-1, r0)
        AQ = np.stack([AM(Qb[:, i].reshape(-1, 6)).reshape(-1) for i in range(k)], axis=1)
        c = np.linalg.lstsq(AQ, r0, rcond=None)[0]
        best = np.linalg.norm(r0 - AQ @ c)
        assert abs(info.history[k] - best) <= 1e-9 * np.linalg.norm(r0), (k, info.history[k], best)


def test_full_gmres_reaches_dense_solution():
    m, K, col = _setup((2, 2, 2), seed=3)
    om = np.array([27.0])
    b = _b(m.n_cells, 2)
    n = 6 * m.n_cells
    x, info = krylov.fgmres(K, m.volume, m.zone, om, b, col, "SGS", restart=n, rtol=1e-14, max_iters=n)
    xd = solve.dense_solve(K, m.volume, m.zone, om, b)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd), info.iters
    assert info.iters <= n


def test_exact_preconditioner_needs_one_iteration():
    m, K, col = _setup()
    Kd = K.copy()
    Kd.offd[:] = 0.0                               # block diagonal: Jacobi's M is A itself
    om = np.array([9.0])
    b = _b(m.n_cells, 4)
    x, info = krylov.fgmres(Kd, m.volume, m.zone, om, b, col, "JACOBI", restart=5, rtol=1e-12)
    assert info.iters == 1 and info.status == solve.OK
    xd = np.linalg.solve(solve.system_diag(Kd, m.volume, m.zone, om), b[..., None])[..., 0]
    assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd)


def test_history_monotone_and_true_residual():
    m, K, col = _setup()
    om = np.array([36.0])
    b = _b(m.n_cells, 5)
    x, info = krylov.fgmres(K, m.volume, m.zone, om, b, col, "DILU", restart=8, rtol=1e-10, max_iters=400)
    assert info.status == solve.OK
    h = np.array(info.history)
    for c0 in range(0, len(h) - 1, 8):             # within each cycle of 8
        seg = h[c0:c0 + 9]
        assert np.all(np.diff(seg) <= 1e-12 * h[0])
    assert abs(info.true_res - info.rel_res) <= 1e-9
    xd = solve.dense_solve(K, m.volume, m.zone, om, b)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)


def test_more_inner_sweeps_fewer_iterations():
    m, K, col = _setup()
    om = np.array([18.0])
    b = _b(m.n_cells, 7)
    _, i1 = krylov.fgmres(K, m.volume, m.zone, om, b, col, "DILU", restart=10, rtol=1e-10, inner_sweeps=1)
    _, i3 = krylov.fgmres(K, m.volume, m.zone, om, b, col, "DILU", restart=10, rtol=1e-10, inner_sweeps=3)
    assert i1.status == solve.OK and i3.status == solve.OK
    assert i3.iters < i1.iters


def test_learned_exact_network_converges_in_one_iteration():
    m, K, col = _setup()
    om = np.array([36.0])
    b = _b(m.n_cells, 8)
    net = lambda r: solve.dense_solve(K, m.volume, m.zone, om, r)
    x, info = krylov.fgmres(K, m.volume, m.zone, om, b, col, "LEARNED", restart=5, rtol=1e-12, net=net)
    assert info.status == solve.OK and info.iters == 1 and info.learned == 1
    xd = solve.dense_solve(K, m.volume, m.zone, om, b)
    assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd)


def test_learned_zero_network_is_dilu():
    m, K, col = _setup()
    om = np.array([18.0])
    b = _b(m.n_cells, 9)
    kw = dict(restart=6, rtol=0.0, max_iters=14, inner_sweeps=2)
    x0, i0 = krylov.fgmres(K, m.volume, m.zone, om, b, col, "DILU", **kw)
    x1, i1 = krylov.fgmres(K, m.volume, m.zone, om, b, col, "LEARNED", net=np.zeros_like, **kw)
    assert i1.learned == 0
    assert np.array_equal(x0, x1) and i0.history == i1.history


class _Scripted:
    """A network that answers with the exact correction (kept) or zero (rejected)
    following a script of True/False per call; counts its calls."""

    def __init__(self, K, m, om, script):
        self.K, self.m, self.om, self.script, self.calls = K, m, om, list(script), 0

    def __call__(self, r):
        good = self.script[self.calls] if self.calls < len(self.script) else True
        self.calls += 1
        if not good:
            return np.zeros_like(r)
        return 0.5 * solve.dense_solve(self.K, self.m.volume, self.m.zone, self.om, r)


def test_learned_controller_switches_off_after_three_rejections():
    m, K, col = _setup()
    om = np.array([18.0])
    b = _b(m.n_cells, 12)
    kw = dict(restart=6, rtol=0.0, max_iters=12, inner_sweeps=1)
    # rejected, rejected, rejected: never evaluated again, although it would now help
    net = _Scripted(K, m, om, [False, False, False])
    x1, i1 = krylov.fgmres(K, m.volume, m.zone, om, b, col, "LEARNED", net=net, **kw)
    x0, i0 = krylov.fgmres(K, m.volume, m.zone, om, b, col, "DILU", **kw)
    assert net.calls == krylov.OFF_AFTER == 3 and i1.switched_off and i1.learned == 0
    assert np.array_equal(x0, x1) and i0.history == i1.history
    # two rejections, then kept steps: the run is broken and the network stays on
    net = _Scripted(K, m, om, [False, False, True, False, False, True])
    _, i2 = krylov.fgmres(K, m.volume, m.zone, om, b, col, "LEARNED", net=net, restart=6, rtol=1e-12,
                          max_iters=6, inner_sweeps=1)
    assert not i2.switched_off and i2.learned >= 1 and net.calls == i2.iters


def test_learned_random_network_reaches_dense_solution():
    m, K, col = _setup()
    om = np.array([18.0])
    b = _b(m.n_cells, 10)
    Ds = solve.system_diag(K, m.volume, m.zone, om)
    w = learned.init_weights(11)
    w[-64 * 12:] *= 10.0
    x, info = krylov.fgmres(K, m.volume, m.zone, om, b, col, "LEARNED", restart=10, rtol=1e-11, max_iters=400,
                            net=lambda r: learned.apply(w, K, Ds, r))
    assert info.status == solve.OK and info.learned >= 1
    xd = solve.dense_solve(K, m.volume, m.zone, om, b)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
