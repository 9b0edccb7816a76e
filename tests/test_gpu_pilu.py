"""GPU parity of the partition-local ILU(0) (kind "pilu": each partition of
set_partitions factored and swept on its own in the natural cell order, the couplings
between partitions left out) against the oracle: Richardson with the natural-order DILU
(every cell its own class, in id order) on the partition_dropped matrix.  Iterates (FP64,
1e-11) on two-colour and general-colouring meshes, partitions whose levels are wider
than a wave and span several 64-position groups, five systems per call (three workgroups
per partition), frozen-turbulence and phase-lagged systems, converged FP32/BF16 solves
against the dense dropped system, the residual history, graph replay, FGMRES, the RK
driver, new partitions, work units and workgroup sizes, single-cell partitions, the kernel
statistics and the error paths."""
import numpy as np
import pytest

from oracle import assemble, rk, solve
from paper_2404_01407_amd import synth

from gpu_helpers import itererr, relerr, to_dev

pytestmark = pytest.mark.gpu

ITER_TOL = 1e-11
OMEGA = np.array([[0.0], [18.0], [36.0]])


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2404_01407_amd import fnlh
    return fnlh


def _case(kind, seed=4, shape=None):
    if kind == "passage":
        m = synth.passage_block(*(shape or (12, 6, 4)), 36, seed=seed)   # two colours
    else:
        m = synth.cascade_block(*(shape or (8, 5, 3)), 36, seed=seed)    # odd pitch
    Q = synth.flow_state(m, seed)
    return m, Q, assemble.assemble(m, Q)


def _rhs(m, seed, n=3):
    return [synth.rhs(m.n_cells, seed + s, real=(s == 0)) for s in range(n)]


def _solve(c, systems, bs, **kw):
    import torch
    xs = [to_dev(np.zeros((c.n, 6), complex)) for _ in systems]
    out = c.relax(systems, xs, [to_dev(b) for b in bs], kind="pilu", **kw)
    torch.cuda.synchronize()
    return (*out, [x.cpu().numpy() for x in xs])


def _natural(m):
    return np.arange(m.n_cells)


def _ctx(F, m, Q, part, storage="f64", omega=OMEGA):
    c = F.Context(m, storage=storage)
    c.assemble_jacobian(to_dev(Q))
    c.set_partitions(part)
    c.set_harmonics(omega)
    return c


def _level_widths(m, part):
    """Rows per level of the natural-order level schedule, over all partitions."""
    n = m.n_cells
    lower = [[] for _ in range(n)]
    for a, b in m.edges:
        if part[a] == part[b]:
            lo, hi = min(a, b), max(a, b)
            lower[hi].append(lo)
    lev = np.zeros(n, np.int64)
    for u in range(n):
        if lower[u]:
            lev[u] = 1 + max(lev[v] for v in lower[u])
    widths = {}
    for u in range(n):
        widths[(part[u], lev[u])] = widths.get((part[u], lev[u]), 0) + 1
    return widths


@pytest.mark.parametrize("mesh", ["passage", "cascade"])
def test_pilu_iterates_match_oracle(F, mesh):
    m, Q, K = _case(mesh)
    part = synth.rcb_partition(m, 37)
    c = _ctx(F, m, Q, part)
    bs = _rhs(m, 0)
    st, rep, xs = _solve(c, [0, 1, 2], bs, max_sweeps=20, rtol=0.0)
    Kd = solve.partition_dropped(K, part)
    for s in range(3):
        x_or, info = solve.richardson(Kd, m.volume, m.zone, OMEGA[s], bs[s], _natural(m), "DILU", rtol=0.0,
                                      max_sweeps=20)
        assert itererr(xs[s], x_or) <= ITER_TOL, (mesh, s, itererr(xs[s], x_or))
        assert abs(rep[s]["rel_res"] - info.rel_res) <= 1e-9 * info.rel_res + 1e-15
        assert rep[s]["sweeps"] == 20
    c.close()


def test_pilu_wide_levels_many_groups_five_systems(F):
    """Partitions of up to 600 cells: levels of more than 64 rows (a wave loops over a
    level), partitions straddling 64-position groups, and five systems (workgroups take
    two, two and one)."""
    m, Q, K = _case("passage", seed=8, shape=(24, 12, 6))
    part = synth.rcb_partition(m, 600)
    widths = _level_widths(m, part)
    assert max(widths.values()) > 64 and np.bincount(part).max() > 64
    om = np.array([[0.0], [9.0], [18.0], [27.0], [36.0]])
    c = _ctx(F, m, Q, part, omega=om)
    bs = _rhs(m, 3, n=5)
    st, rep, xs = _solve(c, [0, 1, 2, 3, 4], bs, max_sweeps=5, rtol=0.0)
    Kd = solve.partition_dropped(K, part)
    for s in (0, 4):
        x_or, _ = solve.richardson(Kd, m.volume, m.zone, om[s], bs[s], _natural(m), "DILU", rtol=0.0, max_sweeps=5)
        assert itererr(xs[s], x_or) <= ITER_TOL, (s, itererr(xs[s], x_or))
    # each system is independent of the others in the call
    _, _, one = _solve(c, [3], [bs[3]], max_sweeps=5, rtol=0.0)
    assert np.array_equal(one[0], xs[3])
    c.close()


def test_pilu_frozen_turbulence(F):
    m, Q, K = _case("passage", seed=5)
    part = synth.rcb_partition(m, 50)
    c = _ctx(F, m, Q, part)
    c.set_frozen_turbulence([0, 1, 1])
    bs = _rhs(m, 7)
    st, rep, xs = _solve(c, [0, 1, 2], bs, max_sweeps=12, rtol=0.0)
    Kd = solve.partition_dropped(K, part)
    for s in range(3):
        f = solve.richardson_frozen if s else solve.richardson
        x_or, _ = f(Kd, m.volume, m.zone, OMEGA[s], bs[s], _natural(m), "DILU", rtol=0.0, max_sweeps=12)
        assert itererr(xs[s], x_or) <= ITER_TOL, (s, itererr(xs[s], x_or))
        if s:
            assert np.all(xs[s][:, 5] == 0)
    c.close()


def test_pilu_phase_lagged(F):
    m = synth.cascade_block(8, 5, 4, 36, seed=11)
    Q = synth.flow_state(m, 11)
    K = assemble.assemble(m, Q)
    sigma = np.array([0.0, 0.7, -1.9])
    part = synth.rcb_partition(m, 40)
    c = _ctx(F, m, Q, part)
    c.set_phase_lag(m.edge_phase, sigma)
    bs = _rhs(m, 9)
    st, rep, xs = _solve(c, [0, 1, 2], bs, max_sweeps=15, rtol=0.0)
    for s in range(3):
        Kp = solve.partition_dropped(solve.phase_lagged(K, m.edge_phase, sigma[s]), part)
        x_or, _ = solve.richardson(Kp, m.volume, m.zone, OMEGA[s], bs[s], _natural(m), "DILU", rtol=0.0,
                                   max_sweeps=15)
        assert itererr(xs[s], x_or) <= ITER_TOL, (s, itererr(xs[s], x_or))
    c.close()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_pilu_converged_reduced_precision(F, storage):
    m, Q, K = _case("passage", seed=6)
    part = synth.rcb_partition(m, 60)
    c = _ctx(F, m, Q, part, storage=storage)
    bs = _rhs(m, 10)
    st, rep, xs = _solve(c, [0, 1, 2], bs, max_sweeps=4000, rtol=1e-11)
    assert st == F.OK, rep
    Kd = solve.partition_dropped(K, part)
    for s in range(3):
        assert relerr(xs[s], solve.dense_solve(Kd, m.volume, m.zone, OMEGA[s], bs[s])) <= 1e-9, (storage, s)
        assert rep[s]["rel_res"] <= 1e-11
    c.close()


def test_pilu_history_and_stop(F):
    """The residual history and the stop rule (the returned x is one sweep past the first
    iterate that met the tolerance) match the oracle's Richardson history."""
    m, Q, K = _case("cascade", seed=2)
    part = synth.rcb_partition(m, 30)
    c = _ctx(F, m, Q, part)
    bs = _rhs(m, 12)
    st, rep, hist, xs = _solve(c, [0, 1, 2], bs, max_sweeps=500, rtol=1e-6, history=True)
    assert st == F.OK
    Kd = solve.partition_dropped(K, part)
    for s in range(3):
        _, info = solve.richardson(Kd, m.volume, m.zone, OMEGA[s], bs[s], _natural(m), "DILU", rtol=1e-6,
                                   max_sweeps=500)
        S = info.sweeps
        assert rep[s]["sweeps"] == S + 1
        np.testing.assert_allclose(hist[s][:S + 1], info.history[:S + 1], rtol=1e-9, atol=1e-14 * info.history[0])
    c.close()


def test_pilu_graph_replay_bitwise(F):
    m, Q, K = _case("passage", seed=3)
    part = synth.rcb_partition(m, 45)
    c = _ctx(F, m, Q, part)
    bs = _rhs(m, 14)
    _, r0, x0 = _solve(c, [0, 1, 2], bs, max_sweeps=40, rtol=1e-7, check_every=8, use_graph=False)
    _, r1, x1 = _solve(c, [0, 1, 2], bs, max_sweeps=40, rtol=1e-7, check_every=8, use_graph=True)
    _, r2, x2 = _solve(c, [0, 1, 2], bs, max_sweeps=40, rtol=1e-7, check_every=8, use_graph=True)
    for s in range(3):
        assert np.array_equal(x0[s], x1[s]) and np.array_equal(x1[s], x2[s])
        assert r0[s]["sweeps"] == r1[s]["sweeps"]
    c.close()


def test_pilu_gmres(F):
    import torch
    m, Q, K = _case("cascade", seed=7)
    part = synth.rcb_partition(m, 25)
    c = _ctx(F, m, Q, part)
    bs = _rhs(m, 30)
    xs = [to_dev(np.zeros((m.n_cells, 6), complex)) for _ in range(3)]
    st, rep = c.gmres([0, 1, 2], xs, [to_dev(b) for b in bs], kind="pilu", restart=10, max_iters=300, rtol=1e-11)
    torch.cuda.synchronize()
    assert st == F.OK, rep
    Kd = solve.partition_dropped(K, part)
    for s in range(3):
        assert relerr(xs[s].cpu().numpy(), solve.dense_solve(Kd, m.volume, m.zone, OMEGA[s], bs[s])) <= 1e-9
    c.close()


def test_pilu_rk_mean_steps(F):
    import torch
    m, Q, K = _case("cascade", seed=9)
    part = synth.rcb_partition(m, 30)
    c = F.Context(m)
    c.set_partitions(part)
    st = to_dev(Q)
    c.assemble_jacobian(st)
    c.set_harmonics(np.zeros((1, m.n_zones)))
    _, hm = c.rk_mean(0, st, 2, kind="pilu", max_sweeps=10, rtol=0.0)
    torch.cuda.synchronize()
    Qm, hmo = Q.copy(), []
    for _ in range(2):
        Qm, r0 = rk.mean_step(m, Qm, _natural(m), rtol=0.0, max_sweeps=10, part=part)
        hmo.append(r0)
    assert relerr(st.cpu().numpy(), Qm) <= 1e-10
    np.testing.assert_allclose(hm, hmo, rtol=1e-11)
    c.close()


def test_pilu_new_partitions_rebuild(F):
    m, Q, K = _case("passage", seed=10)
    p1 = synth.rcb_partition(m, 40)
    p2 = synth.rcb_partition(m, 90)
    c = _ctx(F, m, Q, p1)
    bs = _rhs(m, 40)
    kw = dict(max_sweeps=10, rtol=0.0)
    _, _, a = _solve(c, [0, 1, 2], bs, **kw)
    c.set_partitions(p2)                      # new couplings dropped: the matrix again
    c.assemble_jacobian(to_dev(Q))
    c.set_harmonics(OMEGA)
    _, _, b = _solve(c, [0, 1, 2], bs, **kw)
    for s, (xs, p) in enumerate(((a, p1), (b, p2))):
        Kd = solve.partition_dropped(K, p)
        for j in range(3):
            x_or, _ = solve.richardson(Kd, m.volume, m.zone, OMEGA[j], bs[j], _natural(m), "DILU", **kw)
            assert itererr(xs[j], x_or) <= ITER_TOL, (s, j)
    c.close()


def test_pilu_stats(F):
    m, Q, K = _case("passage", seed=12)
    part = synth.rcb_partition(m, 50)
    c = _ctx(F, m, Q, part)
    c.stats_enable(True)
    bs = _rhs(m, 50)
    st, rep, xs = _solve(c, [0, 1, 2], bs, max_sweeps=9, rtol=0.0, check_every=3)
    s = c.stats()["pilu"]
    # 9 sweeps, then launches in which every system has stopped (the loop reads the
    # stop flags every 3 sweeps)
    assert 9 <= s["launches"] <= 12 and s["total_ms"] > 0 and s["alg_bytes"] > 0
    assert all(r["sweeps"] == 9 for r in rep)
    c.close()


def test_pilu_work_units_bitwise(F):
    """Work units (consecutive partitions swept by one workgroup, levels merged) and the
    workgroup size change the schedule, not the arithmetic: each partition alone, the
    automatic unit and units of up to 400 cells, with 64, 128 and 256 lanes, give the
    same iterates bit for bit."""
    m, Q, K = _case("passage", seed=8, shape=(24, 12, 6))
    part = synth.rcb_partition(m, 40)
    c = _ctx(F, m, Q, part)
    bs = _rhs(m, 70)
    out = []
    for unit, nt in ((1, 0), (0, 64), (0, 128), (400, 256)):
        c.tune(pilu_unit=unit, pilu_threads=nt)
        _, rep, xs = _solve(c, [0, 1, 2], bs, max_sweeps=6, rtol=0.0)
        out.append(xs)
    for xs in out[1:]:
        for s in range(3):
            assert np.array_equal(xs[s], out[0][s])
    Kd = solve.partition_dropped(K, part)
    x_or, _ = solve.richardson(Kd, m.volume, m.zone, OMEGA[2], bs[2], _natural(m), "DILU", rtol=0.0, max_sweeps=6)
    assert itererr(out[2][2], x_or) <= ITER_TOL
    c.close()


def test_pilu_partitions_above_64k_lds(F):
    """Partitions of 1440 cells: FP64 y vectors of 138 KB, more than 64 KiB of LDS."""
    m, Q, K = _case("passage", seed=14, shape=(24, 12, 10))
    part = synth.rcb_partition(m, 1500)
    assert np.bincount(part).max() * 96 > 65536
    c = _ctx(F, m, Q, part)
    bs = _rhs(m, 80)
    st, rep, xs = _solve(c, [1], bs[1:2], max_sweeps=3, rtol=0.0)
    Kd = solve.partition_dropped(K, part)
    x_or, _ = solve.richardson(Kd, m.volume, m.zone, OMEGA[1], bs[1], _natural(m), "DILU", rtol=0.0, max_sweeps=3)
    assert itererr(xs[0], x_or) <= ITER_TOL
    c.close()


def test_pilu_single_cell_partitions(F):
    """One cell per partition: no in-partition couplings (no packed slots at all), the
    dropped matrix is block diagonal and one sweep solves it exactly."""
    m, Q, K = _case("cascade", seed=15)
    part = np.arange(m.n_cells, dtype=np.int32)[::-1].copy()     # labels in any order
    c = _ctx(F, m, Q, part)
    bs = _rhs(m, 90)
    st, rep, xs = _solve(c, [0, 1, 2], bs, max_sweeps=1, rtol=0.0)
    for s in range(3):
        Ds = solve.system_diag(K, m.volume, m.zone, OMEGA[s])
        xd = np.linalg.solve(Ds, bs[s][..., None])[..., 0]
        assert relerr(xs[s], xd) <= 1e-12, s
        assert rep[s]["rel_res"] <= 1e-12
    c.close()


def test_pilu_errors(F):
    m, Q, K = _case("passage", seed=13)
    c = F.Context(m)
    c.assemble_jacobian(to_dev(Q))
    c.set_harmonics(OMEGA)
    bs = _rhs(m, 60)
    with pytest.raises(F.FnlhError):          # no partitions
        _solve(c, [0], bs[:1], max_sweeps=3, rtol=0.0)
    c.close()
    big, Qb, _ = _case("passage", seed=13, shape=(24, 12, 30))
    c = _ctx(F, big, Qb, synth.rcb_partition(big, 4500), storage="f32")   # 4320 cells: 207 KB of y
    with pytest.raises(F.FnlhError):          # a partition larger than a workgroup's LDS holds
        _solve(c, [0], [synth.rhs(big.n_cells, 1)], max_sweeps=3, rtol=0.0)
    c.close()
    # the batched relax takes DILU, SGS and the learned kind only
    c = _ctx(F, m, Q, synth.rcb_partition(m, 40))
    B = F.Batch([c])
    x = to_dev(np.zeros((m.n_cells, 6), complex))
    with pytest.raises(F.FnlhError):
        B.relax([[0]], [[x]], [[to_dev(bs[0])]], kind="pilu", max_sweeps=3, rtol=0.0)
    B.close()
    c.close()
