"""Batched solves of many independent instances against the same instances solved one
by one (bitwise: the batched launch runs the same per-tile arithmetic) and against the
oracle."""
import numpy as np
import pytest

from oracle import assemble, solve
from paper_2404_01407_amd import synth

from gpu_helpers import relerr, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    from paper_2404_01407_amd import fnlh
    return fnlh


def _instances(F, storage, specs):
    out = []
    for (shape, nb, nh, seed) in specs:
        m = synth.passage_block(*shape, nb, seed=seed) if shape[0] > 0 else synth.multi_row(4, 6, 3, seed=seed)
        Q = synth.flow_state(m, seed)
        c = F.Context(m, storage=storage)
        c.assemble_jacobian(to_dev(Q))
        om = synth.omegas_single_zone(nh, nb) if m.n_zones == 1 else synth.omegas_multi_row(nh)
        c.set_harmonics(om)
        bs = [synth.rhs(m.n_cells, 50 + s, real=(s == 0)) for s in range(nh + 1)]
        out.append((m, Q, c, om, bs))
    return out


SPECS = [((9, 6, 5), 24, 1, 1), ((12, 7, 6), 40, 3, 2), ((6, 5, 4), 60, 8, 3), ((15, 8, 8), 33, 4, 4),
         ((7, 7, 3), 50, 2, 5), ((0, 0, 0), 36, 2, 6)]


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_per_instance(F, storage, graph):
    import torch
    insts = _instances(F, storage, SPECS)
    B = F.Batch([c for (_, _, c, _, _) in insts])
    systems = [list(range(len(bs))) for (_, _, _, _, bs) in insts]
    xs = [[torch.zeros((m.n_cells, 6), dtype=torch.complex128, device="cuda") for _ in bs] for (m, _, _, _, bs) in insts]
    bd = [[to_dev(b) for b in bs] for (_, _, _, _, bs) in insts]
    st, reps = B.relax(systems, xs, bd, kind="dilu", max_sweeps=2000, rtol=1e-9, check_every=8, use_graph=graph)
    assert st == 0
    for i, (m, Q, c, om, bs) in enumerate(insts):
        xi = [torch.zeros((m.n_cells, 6), dtype=torch.complex128, device="cuda") for _ in bs]
        st1, rep1 = c.relax(systems[i], xi, [to_dev(b) for b in bs], kind="dilu", max_sweeps=2000, rtol=1e-9,
                            check_every=8)
        for j in range(len(bs)):
            a, b = xs[i][j].cpu().numpy(), xi[j].cpu().numpy()
            assert np.array_equal(a, b), (i, j)
            assert reps[i][j]["sweeps"] == rep1[j]["sweeps"]
            assert reps[i][j]["rel_res"] <= 1e-9
    # one instance against the oracle's dense solve
    m, Q, c, om, bs = insts[1]
    K = assemble.assemble(m, Q)
    xd = solve.dense_solve(K, m.volume, m.zone, om[2], bs[2])
    tol = 1e-7 if storage == "f64" else 1e-7
    assert relerr(xs[1][2].cpu().numpy(), xd) <= tol
    B.close()
    for (_, _, c, _, _) in insts:
        c.close()


def test_batch_repeated_solves_graph(F):
    import torch
    insts = _instances(F, "f32", SPECS[:4])
    B = F.Batch([c for (_, _, c, _, _) in insts])
    systems = [list(range(len(bs))) for (_, _, _, _, bs) in insts]
    bd = [[to_dev(b) for b in bs] for (_, _, _, _, bs) in insts]
    ref = None
    for rep in range(3):
        xs = [[torch.zeros((m.n_cells, 6), dtype=torch.complex128, device="cuda") for _ in bs] for (m, _, _, _, bs) in insts]
        st, reps = B.relax(systems, xs, bd, kind="dilu", max_sweeps=2000, rtol=1e-8, check_every=16, use_graph=True)
        got = [[x.cpu().numpy() for x in row] for row in xs]
        if ref is None:
            ref = got
        else:
            for r1, r2 in zip(ref, got):
                for a, b in zip(r1, r2):
                    assert np.array_equal(a, b)
        torch.cuda.synchronize()
    B.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_batch_learned_converges(F, storage):
    """Learned corrections in the batched solver: every instance carries a network with
    the same weights (the network is local per edge, so one set of weights serves every
    mesh); the batched instances and the one solved alone all reach the tolerance, and
    the corrections are counted."""
    import torch
    insts = _instances(F, storage, SPECS)
    nets = []
    w = synth.he_init(3)
    for (_, _, c, _, _) in insts:
        net = F.Network(c)
        net.set_weights(w)
        nets.append(net)
    B = F.Batch([c for (_, _, c, _, _) in insts])
    systems = [list(range(len(bs))) for (_, _, _, _, bs) in insts]
    xs = [[torch.zeros((m.n_cells, 6), dtype=torch.complex128, device="cuda") for _ in bs] for (m, _, _, _, bs) in insts]
    bd = [[to_dev(b) for b in bs] for (_, _, _, _, bs) in insts]
    st, reps = B.relax(systems, xs, bd, kind="learned", max_sweeps=3000, rtol=1e-9, check_every=8, use_graph=True,
                       learn_every=16)
    torch.cuda.synchronize()
    assert st == 0, reps
    steps = 0
    for i, (m, Q, c, om, bs) in enumerate(insts):
        for j in range(len(bs)):
            assert reps[i][j]["rel_res"] <= 1e-9, (i, j, reps[i][j])
            steps += reps[i][j]["learned"] + reps[i][j]["fallbacks"]
            r = torch.empty_like(xs[i][j])
            n2 = c.residual(j, xs[i][j], bd[i][j], r)
            assert np.sqrt(n2) <= 1e-9 * reps[i][j]["res0"] * 1.0001
    assert steps > 0
    B.close()
    for net in nets:
        net.close()
    for (_, _, c, _, _) in insts:
        c.close()


@pytest.mark.parametrize("loop_cells", [0, 300, 10**9])
def test_batch_loop_cells_schedule(F, loop_cells):
    """Instances at or above loop_cells are iterated alone inside the batched call, the
    rest share the launches; every schedule gives the per-instance results bitwise."""
    import torch
    insts = _instances(F, "f32", SPECS[:5])
    B = F.Batch([c for (_, _, c, _, _) in insts])
    B.set_loop_cells(loop_cells)
    systems = [list(range(len(bs))) for (_, _, _, _, bs) in insts]
    xs = [[torch.zeros((m.n_cells, 6), dtype=torch.complex128, device="cuda") for _ in bs] for (m, _, _, _, bs) in insts]
    bd = [[to_dev(b) for b in bs] for (_, _, _, _, bs) in insts]
    st, reps = B.relax(systems, xs, bd, kind="dilu", max_sweeps=2000, rtol=1e-9, check_every=8, use_graph=True)
    assert st == 0
    for i, (m, Q, c, om, bs) in enumerate(insts):
        xi = [torch.zeros((m.n_cells, 6), dtype=torch.complex128, device="cuda") for _ in bs]
        c.relax(systems[i], xi, [to_dev(b) for b in bs], kind="dilu", max_sweeps=2000, rtol=1e-9, check_every=8)
        for j in range(len(bs)):
            assert np.array_equal(xs[i][j].cpu().numpy(), xi[j].cpu().numpy()), (loop_cells, i, j)
    B.close()
    for (_, _, c, _, _) in insts:
        c.close()


@pytest.mark.parametrize("shape", ["hex", "three_row"])
def test_autotune_picks_a_timed_configuration(F, shape):
    """fnlh_autotune times whole solves to the tolerance over path (three-row mesh: two
    colours plus remainder, general), kernel shape and workgroup mapping; the pick is no
    slower than the default configuration it timed, stays on the context, and the solve
    with it reaches the same solution (to the tolerance) as the default one."""
    import torch
    if shape == "hex":
        m = synth.passage_block(12, 8, 6, 36, seed=9)
        om = synth.omegas_single_zone(2, 36)
    else:
        m = synth.multi_row(6, 8, 4, n_blades=(36, 60, 48), seed=5)
        om = synth.omegas_multi_row(2, (36, 60, 48))
    Q = synth.flow_state(m, 9)
    bs = [to_dev(synth.rhs(m.n_cells, 20 + s, real=(s == 0))) for s in range(3)]
    sols = []
    for tuned in (False, True):
        c = F.Context(m, storage="f32")
        c.assemble_jacobian(to_dev(Q))
        c.set_harmonics(om)
        if tuned:
            r = c.autotune(3, rtol=1e-9, max_sweeps=3000)
            n_paths = 2 if shape == "three_row" else 1
            assert r["candidates"] == n_paths * 8 and not r["cached"]  # 3 systems: 1-2 lanes per row
            assert 0 < r["ms_best"] <= r["ms_default"] and r["sweeps"] > 0
            assert r["hybrid"] in ((0, 1) if shape == "three_row" else (1,))
        xs = [torch.zeros_like(b) for b in bs]
        st, rep = c.relax([0, 1, 2], xs, bs, kind="dilu", max_sweeps=3000, rtol=1e-9, use_graph=True)
        assert st == 0 and all(q["rel_res"] <= 1e-9 for q in rep)
        sols.append([x.cpu().numpy() for x in xs])
        c.close()
    K = assemble.assemble(m, Q)
    for s in range(3):
        xd = solve.dense_solve(K, m.volume, m.zone, om[s], bs[s].cpu().numpy())
        for x in (sols[0][s], sols[1][s]):
            assert relerr(x, xd) <= 1e-7


def test_batch_autotune_picks_a_schedule(F):
    """fnlh_batch_autotune times the batched solve for each size threshold, keeps the
    fastest and leaves its solution in x: bitwise the per-instance solves (every schedule
    gives them)."""
    import torch
    insts = _instances(F, "f32", SPECS)
    B = F.Batch([c for (_, _, c, _, _) in insts])
    systems = [list(range(len(bs))) for (_, _, _, _, bs) in insts]
    xs = [[torch.full((m.n_cells, 6), 7.0, dtype=torch.complex128, device="cuda") for _ in bs]
          for (m, _, _, _, bs) in insts]
    bd = [[to_dev(b) for b in bs] for (_, _, _, _, bs) in insts]
    cands = (0, 300, 1 << 40)
    st, pick, ms = B.autotune(systems, xs, bd, candidates=cands, rtol=1e-9, check_every=8)
    assert st == 0 and pick in (0, 300, 1 << 40) and all(ms[k] > 0 for k in cands)
    assert ms[pick] == min(ms.values())
    for i, (m, Q, c, om, bs) in enumerate(insts):
        xi = [torch.zeros((m.n_cells, 6), dtype=torch.complex128, device="cuda") for _ in bs]
        c.relax(systems[i], xi, [to_dev(b) for b in bs], kind="dilu", max_sweeps=5000, rtol=1e-9, check_every=8)
        for j in range(len(bs)):
            assert np.array_equal(xs[i][j].cpu().numpy(), xi[j].cpu().numpy()), (i, j)
    B.close()
    for (_, _, c, _, _) in insts:
        c.close()
