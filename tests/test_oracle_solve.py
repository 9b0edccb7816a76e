"""Pins of the oracle's shifted systems, preconditioners and iteration (no GPU):
dense direct solves, brute-force dense iterates, the DILU / ILU(0) defining
properties, exactness cases, omega = 0, conjugate symmetry, the real 2x2 block form,
linearity, relabelling invariance, divergence detection and the paper's qualitative
convergence claims."""
import numpy as np
import pytest

from oracle import assemble, ordering, solve
from paper_2404_01407_amd import synth


def _case(shape=(4, 3, 2), seed=11, sigma=50.0, jitter=0.1):
    m = synth.passage_block(*shape, 36, seed=seed, jitter=jitter)
    Q = synth.flow_state(m, seed)
    K = assemble.assemble(m, Q, sigma=sigma)
    return m, K


def _dense_perm(K, m, om, colour):
    """Dense K_s permuted to colour-major order (ties by id) and the permutation."""
    A = solve.dense(K, m.volume, m.zone, om)
    order = np.lexsort((np.arange(K.n), colour))
    idx = (6 * order[:, None] + np.arange(6)).reshape(-1)
    return A[np.ix_(idx, idx)], order, idx


def _blocks_lower_upper(Ap, n):
    L = np.zeros_like(Ap)
    U = np.zeros_like(Ap)
    D = np.zeros_like(Ap)
    for i in range(n):
        for k in range(n):
            blk = Ap[6 * i:6 * i + 6, 6 * k:6 * k + 6]
            (L if k < i else U if k > i else D)[6 * i:6 * i + 6, 6 * k:6 * k + 6] = blk
    return L, D, U


@pytest.fixture(scope="module")
def cfg1():
    m = synth.passage_block(16, 8, 4, 36, seed=1)
    Q = synth.flow_state(m, 1)
    K = assemble.assemble(m, Q)
    col = ordering.bipartite_colouring(m.n_cells, m.edges)
    om = synth.omegas_single_zone(1)
    return m, K, col, om


def test_dense_agreement_cfg1(cfg1):
    m, K, col, om = cfg1
    for s in range(2):
        b = synth.rhs(m.n_cells, s, real=(s == 0))
        x, info = solve.richardson(K, m.volume, m.zone, om[s], b, col, "DILU", rtol=1e-13, max_sweeps=400)
        xd = solve.dense_solve(K, m.volume, m.zone, om[s], b)
        assert info.status == solve.OK
        assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= 1e-10


@pytest.mark.parametrize("shape", [(2, 2, 2), (4, 3, 2)])
@pytest.mark.parametrize("kind", ["DILU", "SGS", "JACOBI"])
def test_iterates_match_dense_definition(shape, kind):
    # x^{m+1} = x^m + M^-1 r^m with M formed densely from its definition
    m, K = _case(shape)
    col = ordering.greedy_colouring(m.n_cells, m.edges)
    om = np.array([18.0])
    b = synth.rhs(m.n_cells, 1)
    Ap, order, idx = _dense_perm(K, m, om, col)
    n = K.n
    L, D, U = _blocks_lower_upper(Ap, n)
    if kind == "JACOBI":
        M = D
    else:
        if kind == "SGS":
            Dt = D
        else:
            f = solve.factor(K, m.volume, m.zone, om, col, "DILU")
            Dt = np.zeros_like(Ap)
            for p, i in enumerate(order):
                Dt[6 * p:6 * p + 6, 6 * p:6 * p + 6] = f.Dt[i]
        M = (Dt + L) @ np.linalg.solve(Dt, Dt + U)
    its = []
    solve.richardson(K, m.volume, m.zone, om, b, col, kind, rtol=0.0, max_sweeps=15, iterates=its)
    bp = b.reshape(-1)[idx]
    x = np.zeros_like(bp)
    for it in range(1, 16):
        x = x + np.linalg.solve(M, bp - Ap @ x)
        got = its[it].reshape(-1)[idx]
        assert np.linalg.norm(got - x) <= 1e-12 * np.linalg.norm(x)


def test_dilu_defining_property():
    # diag blocks of M = (Dt+L) Dt^-1 (Dt+U) equal those of K_s; on a triangle-free
    # graph M also equals K_s on every off-diagonal coupling of the pattern
    m, K = _case((4, 3, 3))
    assert not ordering.has_triangle(m.n_cells, m.edges)
    col = ordering.bipartite_colouring(m.n_cells, m.edges)
    om = np.array([36.0])
    f = solve.factor(K, m.volume, m.zone, om, col, "DILU")
    Ap, order, idx = _dense_perm(K, m, om, col)
    L, D, U = _blocks_lower_upper(Ap, K.n)
    Dt = np.zeros_like(Ap)
    for p, i in enumerate(order):
        Dt[6 * p:6 * p + 6, 6 * p:6 * p + 6] = f.Dt[i]
    M = (Dt + L) @ np.linalg.solve(Dt, Dt + U)
    pattern = np.abs(Ap) > 0
    for p in range(K.n):
        pattern[6 * p:6 * p + 6, 6 * p:6 * p + 6] = True
    np.testing.assert_allclose(M[pattern], Ap[pattern], rtol=0, atol=1e-12 * np.abs(Ap).max())


def test_dilu_defining_property_with_triangles():
    """diag(M) = diag(K_s) for M = (Dt+L) Dt^-1 (Dt+U) holds on any graph: it defines
    Dt.  Pinned here on a two-row mesh whose interface edges form triangles (greedy
    colouring, several colours, per-row frequencies), the case of the three-row sector
    and the general-colouring kernels, where DILU and ILU(0) differ.  M - K_s is then
    exactly the strictly off-diagonal part of L Dt^-1 U: the fill DILU leaves out."""
    m = synth.multi_row(3, 4, 2, n_blades=(36, 60), seed=3)
    Q = synth.flow_state(m, 3)
    K = assemble.assemble(m, Q)
    assert ordering.has_triangle(m.n_cells, m.edges)
    col = ordering.greedy_colouring(m.n_cells, m.edges)
    assert col.max() + 1 >= 3
    for om in (np.array([18.0, 30.0]), np.array([0.0, 0.0]), np.array([-54.0, 90.0])):
        f = solve.factor(K, m.volume, m.zone, om, col, "DILU")
        Ap, order, idx = _dense_perm(K, m, om, col)
        n = K.n
        L, D, U = _blocks_lower_upper(Ap, n)
        Dt = np.zeros_like(Ap)
        for p, i in enumerate(order):
            Dt[6 * p:6 * p + 6, 6 * p:6 * p + 6] = f.Dt[i]
        M = (Dt + L) @ np.linalg.solve(Dt, Dt + U)
        scale = np.abs(Ap).max()
        diag = np.zeros_like(Ap, dtype=bool)
        for p in range(n):
            diag[6 * p:6 * p + 6, 6 * p:6 * p + 6] = True
        np.testing.assert_allclose(M[diag], Ap[diag], rtol=0, atol=1e-12 * scale)
        fill = L @ np.linalg.solve(Dt, U)
        fill[diag] = 0.0
        np.testing.assert_allclose(M - Ap, fill, rtol=0, atol=1e-12 * scale)
        # a wrong Dt (one block perturbed) breaks the property
        Dt2 = Dt.copy()
        Dt2[6 * (n // 2):6 * (n // 2) + 6, 6 * (n // 2):6 * (n // 2) + 6] *= 1.001
        M2 = (Dt2 + L) @ np.linalg.solve(Dt2, Dt2 + U)
        assert np.abs(M2[diag] - Ap[diag]).max() > 1e-6 * scale


def test_ilu0_defining_property_with_triangles():
    m = synth.multi_row(3, 4, 2, n_blades=(36, 60), seed=3)
    Q = synth.flow_state(m, 3)
    K = assemble.assemble(m, Q)
    assert ordering.has_triangle(m.n_cells, m.edges)
    col = ordering.greedy_colouring(m.n_cells, m.edges)
    om = np.array([18.0, 30.0])
    f = solve.factor(K, m.volume, m.zone, om, col, "ILU0")
    # dense check: L^ U^ agrees with K_s on the pattern (incl. the diagonal)
    Ap, order, idx = _dense_perm(K, m, om, col)
    n = K.n
    pos = f.pos
    Lh = np.eye(6 * n, dtype=complex)
    Uh = np.zeros((6 * n, 6 * n), complex)
    for (i, k), blk in f.ilu.items():
        pi, pk = pos[i], pos[k]
        if pk < pi:
            Lh[6 * pi:6 * pi + 6, 6 * pk:6 * pk + 6] = blk
        else:
            Uh[6 * pi:6 * pi + 6, 6 * pk:6 * pk + 6] = blk
    LU = Lh @ Uh
    pattern = np.abs(Ap) > 0
    for p in range(n):
        pattern[6 * p:6 * p + 6, 6 * p:6 * p + 6] = True
    np.testing.assert_allclose(LU[pattern], Ap[pattern], rtol=0, atol=1e-11 * np.abs(Ap).max())
    # with triangles DILU differs from ILU(0)
    fd = solve.factor(K, m.volume, m.zone, om, col, "DILU")
    Udiag = np.array([f.ilu[(i, i)] for i in range(n)])
    assert np.abs(Udiag - fd.Dt).max() > 1e-8 * np.abs(fd.Dt).max()


def test_ilu0_equals_dilu_on_hex():
    m, K = _case((4, 3, 2))
    col = ordering.bipartite_colouring(m.n_cells, m.edges)
    om = np.array([18.0])
    b = synth.rhs(m.n_cells, 2)
    a, b_ = [], []
    solve.richardson(K, m.volume, m.zone, om, b, col, "ILU0", rtol=0, max_sweeps=8, iterates=a)
    solve.richardson(K, m.volume, m.zone, om, b, col, "DILU", rtol=0, max_sweeps=8, iterates=b_)
    for u, v in zip(a, b_):
        assert np.linalg.norm(u - v) <= 1e-12 * max(1.0, np.linalg.norm(v))


@pytest.mark.parametrize("kind", ["ILU0", "DILU"])
def test_chain_natural_order_is_exact(kind):
    # block-tridiagonal in natural order has no fill: ILU(0) = LU, one step is exact
    m = synth.chain(12)
    Q = synth.flow_state(m, 3)
    K = assemble.assemble(m, Q)
    col = ordering.natural_colouring(m.n_cells)
    om = np.array([18.0])
    b = synth.rhs(m.n_cells, 1)
    x, info = solve.richardson(K, m.volume, m.zone, om, b, col, kind, rtol=0, max_sweeps=1)
    xd = solve.dense_solve(K, m.volume, m.zone, om, b)
    assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd)


@pytest.mark.parametrize("kind", ["JACOBI", "DILU", "SGS"])
def test_block_diagonal_one_step_exact(kind):
    # explicit scheme K = P: block diagonal, inverted point by point in one step
    m = synth.passage_block(4, 3, 2, 36, seed=2)
    Q = synth.flow_state(m, 2)
    K = assemble.assemble(m, Q, scheme="explicit")
    col = ordering.bipartite_colouring(m.n_cells, m.edges)
    om = np.array([18.0])
    b = synth.rhs(m.n_cells, 1)
    x, _ = solve.richardson(K, m.volume, m.zone, om, b, col, kind, rtol=0, max_sweeps=1)
    xd = solve.dense_solve(K, m.volume, m.zone, om, b)
    assert np.linalg.norm(x - xd) <= 1e-13 * np.linalg.norm(xd)


def test_omega_zero_reproduces_mean(cfg1):
    # K real: with omega = 0 a complex RHS splits into two real mean solves
    m, K, col, om = cfg1
    b = synth.rhs(m.n_cells, 3)
    z = np.array([0.0])
    it_c, it_r, it_i = [], [], []
    solve.richardson(K, m.volume, m.zone, z, b, col, "DILU", rtol=0, max_sweeps=20, iterates=it_c)
    solve.richardson(K, m.volume, m.zone, z, b.real, col, "DILU", rtol=0, max_sweeps=20, iterates=it_r)
    solve.richardson(K, m.volume, m.zone, z, b.imag, col, "DILU", rtol=0, max_sweeps=20, iterates=it_i)
    for c, r, i in zip(it_c, it_r, it_i):
        assert np.linalg.norm(c - (r + 1j * i)) <= 1e-13 * max(1.0, np.linalg.norm(c))
        assert np.abs(r.imag).max() == 0.0


def test_conjugate_symmetry(cfg1):
    # K real: (K - i w V) conj(x) = conj(b), for iterates and the converged solution
    m, K, col, om = cfg1
    b = synth.rhs(m.n_cells, 1)
    a1, a2 = [], []
    x1, _ = solve.richardson(K, m.volume, m.zone, om[1], b, col, "DILU", rtol=1e-12, max_sweeps=300, iterates=a1)
    x2, _ = solve.richardson(K, m.volume, m.zone, -om[1], np.conj(b), col, "DILU", rtol=1e-12, max_sweeps=300, iterates=a2)
    assert len(a1) == len(a2)
    for u, v in zip(a1, a2):
        assert np.linalg.norm(u - np.conj(v)) <= 1e-13 * max(1.0, np.linalg.norm(u))
    xd = solve.dense_solve(K, m.volume, m.zone, -om[1], np.conj(b))
    assert np.linalg.norm(np.conj(x1) - xd) <= 1e-9 * np.linalg.norm(xd)


def test_real_block_form():
    # the paper's equivalent real system [[A, -W], [W, A]] [Re x; Im x] = [Re B; Im B]
    m, K = _case((4, 3, 2))
    om = np.array([54.0])
    b = synth.rhs(m.n_cells, 5)
    n6 = 6 * K.n
    Areal = solve.dense(K, m.volume, m.zone, np.array([0.0])).real
    W = np.diag(np.repeat(om[0] * m.volume, 6))
    big = np.block([[Areal, -W], [W, Areal]])
    sol = np.linalg.solve(big, np.concatenate([b.real.reshape(-1), b.imag.reshape(-1)]))
    xc = solve.dense_solve(K, m.volume, m.zone, om, b).reshape(-1)
    np.testing.assert_allclose(sol[:n6] + 1j * sol[n6:], xc, rtol=0, atol=1e-10 * np.abs(xc).max())
    col = ordering.bipartite_colouring(m.n_cells, m.edges)
    x, _ = solve.richardson(K, m.volume, m.zone, om, b, col, "DILU", rtol=1e-13, max_sweeps=500)
    assert np.linalg.norm(x.reshape(-1) - (sol[:n6] + 1j * sol[n6:])) <= 1e-10 * np.linalg.norm(xc)


def test_linearity(cfg1):
    m, K, col, om = cfg1
    b1 = synth.rhs(m.n_cells, 1)
    b2 = synth.rhs(m.n_cells, 2)
    al = 0.7 - 0.3j
    a, b_, c = [], [], []
    solve.richardson(K, m.volume, m.zone, om[1], b1, col, "DILU", rtol=0, max_sweeps=10, iterates=a)
    solve.richardson(K, m.volume, m.zone, om[1], b2, col, "DILU", rtol=0, max_sweeps=10, iterates=b_)
    solve.richardson(K, m.volume, m.zone, om[1], b1 + al * b2, col, "DILU", rtol=0, max_sweeps=10, iterates=c)
    for u, v, w in zip(a, b_, c):
        assert np.linalg.norm(w - (u + al * v)) <= 1e-12 * max(1.0, np.linalg.norm(w))


def test_relabelling_invariance():
    m, K = _case((4, 3, 2), seed=9)
    Q = synth.flow_state(m, 9)
    rng = np.random.default_rng(5)
    p = rng.permutation(m.n_cells)                  # old id -> new id
    inv = np.argsort(p)
    e2 = p[m.edges]
    K2 = assemble.residual_jacobian(Q[inv], e2, m.area, p[m.bface_cell], m.bface_area)
    K2 = assemble.preconditioner_matrix(K2)
    col = ordering.bipartite_colouring(m.n_cells, m.edges)
    col2 = col[inv]
    om = np.array([18.0])
    b = synth.rhs(m.n_cells, 1)
    x1, _ = solve.richardson(K, m.volume, m.zone, om, b, col, "DILU", rtol=0, max_sweeps=12)
    x2, _ = solve.richardson(K2, m.volume[inv], m.zone[inv], om, b[inv], col2, "DILU", rtol=0, max_sweeps=12)
    assert np.linalg.norm(x2 - x1[inv]) <= 1e-13 * np.linalg.norm(x1)


def test_divergence_detected():
    # off-diagonal couplings tripled: block Jacobi's iteration matrix has spectral
    # radius > 1 and the residual grows past 1e3 times its initial value
    m, K = _case((4, 3, 2))
    K.offd *= 3.0
    col = ordering.bipartite_colouring(m.n_cells, m.edges)
    b = synth.rhs(m.n_cells, 1)
    x, info = solve.richardson(K, m.volume, m.zone, np.array([0.0]), b, col, "JACOBI", rtol=1e-8, max_sweeps=2000)
    assert info.status == solve.DIVERGED


def test_paper_mode_limits(cfg1):
    m, K, col, om = cfg1
    b = synth.rhs(m.n_cells, 1)
    x, info = solve.paper_mode(K, m.volume, m.zone, om[1], b, col)
    assert info.sweeps <= 10
    assert info.status == solve.OK and info.rel_res <= 1e-2


def test_qualitative_claims(cfg1):
    """In kind, on the linear solve: (Q2) higher frequency converges no slower,
    (Q3) a smaller CFL number gives better diagonal dominance and fewer linear sweeps,
    (Q4) the implicit ILU-type solve needs fewer sweeps than block Jacobi."""
    m, K, col, om = cfg1
    Q = synth.flow_state(m, 1)
    b = synth.rhs(m.n_cells, 1)
    sweeps_w = []
    for w in (0.0, 18.0, 36.0, 54.0):
        _, info = solve.richardson(K, m.volume, m.zone, np.array([w]), b, col, "DILU", rtol=1e-8, max_sweeps=2000)
        sweeps_w.append(info.sweeps)
    assert all(a >= c for a, c in zip(sweeps_w, sweeps_w[1:])), sweeps_w
    sweeps_s = []
    for sg in (10.0, 20.0, 50.0, 100.0):
        Ks = assemble.assemble(m, Q, sigma=sg)
        _, info = solve.richardson(Ks, m.volume, m.zone, np.array([18.0]), b, col, "DILU", rtol=1e-8, max_sweeps=2000)
        sweeps_s.append(info.sweeps)
    assert all(a <= c for a, c in zip(sweeps_s, sweeps_s[1:])), sweeps_s
    _, ij = solve.richardson(K, m.volume, m.zone, np.array([18.0]), b, col, "JACOBI", rtol=1e-8, max_sweeps=2000)
    assert sweeps_w[1] < ij.sweeps
