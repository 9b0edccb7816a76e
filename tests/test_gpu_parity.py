"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on the same
seeded inputs.

Tolerances (FP64 mode): the device sums in a different order than NumPy (fused
two-colour pass, Gauss-Jordan instead of LAPACK inverses), so iterates differ by
rounding only; the iteration is a contraction (rho ~ 0.7), so the difference after m
sweeps stays at a small multiple of machine epsilon times the iterate.  1e-11 relative
leaves three orders of margin over the observed ~1e-14.  Converged solutions are held
to the spec bar: relative residual <= 1e-10 and agreement with a dense direct
solve to 1e-9."""
import numpy as np
import pytest

from oracle import assemble, ordering, precision, solve
from paper_2404_01407_amd import synth

from gpu_helpers import blocks_user_layout, case, itererr, relerr, rounded, to_dev

pytestmark = pytest.mark.gpu

ITER_TOL = 1e-11


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2404_01407_amd import fnlh
    return fnlh


def _ctx(F, m, Q, storage="f64", outer="exact", ordering_="auto", user_colour=None, sigma=50.0, scheme="implicit",
         factor_slots=0):
    c = F.Context(m, storage=storage, outer=outer, ordering=ordering_, user_colour=user_colour,
                  factor_slots=factor_slots)
    c.assemble_jacobian(to_dev(Q), eps=0.6, sigma=sigma, scheme=scheme)
    return c


def _solve(c, systems, bs, x0s=None, **kw):
    import torch
    xs = [to_dev(np.zeros((c.n, 6), complex) if x0s is None else x0s[j]) for j in range(len(systems))]
    bd = [to_dev(b.astype(complex)) for b in bs]
    st, rep = c.relax(systems, xs, bd, **kw)
    torch.cuda.synchronize()
    return st, rep, [x.cpu().numpy() for x in xs]


def test_assembly_matches_oracle(F):
    m, Q, K = case()
    for storage in ("f64", "f32", "bf16"):
        c = _ctx(F, m, Q, storage=storage)
        d, o = c.get_blocks()
        d, o = d.cpu().numpy(), o.cpu().numpy()
        Kr = rounded(K, storage)
        dref, oref = blocks_user_layout(Kr)
        if storage == "f64":
            scale = np.abs(dref).max()
            assert np.abs(d - dref).max() <= 1e-13 * scale
            assert np.abs(o - oref).max() <= 1e-13 * scale
        else:
            # both sides round their FP64 entry to nearest-even.  The FP64 entries
            # differ by summation-order rounding (~1e-16 of the block scale; entries that
            # cancel to zero, such as the off-identity part of a closed cell's diagonal,
            # are pure rounding noise), so allow one storage ulp plus that FP64 noise
            ulp = 2.0 ** -23 if storage == "f32" else 2.0 ** -7
            for got, ref in ((d, dref), (o, oref)):
                scale = np.abs(ref).reshape(ref.shape[0], -1).max(axis=1)
                scale = scale.reshape((-1,) + (1,) * (ref.ndim - 1))
                tol = ulp * np.abs(ref) + 1e-13 * scale
                assert np.all(np.abs(got - ref) <= tol)
                big = np.abs(ref) > 1e-10 * scale
                assert np.mean(got[big] == ref[big]) > 0.999
        c.close()


@pytest.mark.parametrize("kind", ["dilu", "sgs", "jacobi"])
def test_iterates_cfg1(F, kind):
    m, Q, K = case()
    c = _ctx(F, m, Q)
    om = synth.omegas_single_zone(1)
    c.set_harmonics(om)
    col, nc = c.ordering()
    assert nc == 2
    bs = [synth.rhs(m.n_cells, 0, real=True), synth.rhs(m.n_cells, 1)]
    st, rep, xs = _solve(c, [0, 1], bs, kind=kind, max_sweeps=50, rtol=0.0)
    for s in range(2):
        x_or, info = solve.richardson(K, m.volume, m.zone, om[s], bs[s], col, kind.upper(), rtol=0.0, max_sweeps=50)
        assert rep[s]["sweeps"] == 50
        assert itererr(xs[s], x_or) <= ITER_TOL, (kind, s, itererr(xs[s], x_or))
        assert abs(rep[s]["rel_res"] - info.rel_res) <= 1e-9 * info.rel_res + 1e-15
    c.close()


def test_converged_vs_dense_cfg1(F):
    m, Q, K = case()
    c = _ctx(F, m, Q)
    om = synth.omegas_single_zone(1)
    c.set_harmonics(om)
    bs = [synth.rhs(m.n_cells, 0, real=True), synth.rhs(m.n_cells, 1)]
    st, rep, xs = _solve(c, [0, 1], bs, kind="dilu", max_sweeps=1000, rtol=1e-12)
    assert st == 0
    for s in range(2):
        xd = solve.dense_solve(K, m.volume, m.zone, om[s], bs[s])
        assert rep[s]["rel_res"] <= 1e-10
        assert relerr(xs[s], xd) <= 1e-9
        r = bs[s] - solve.apply(K, solve.system_diag(K, m.volume, m.zone, om[s]), xs[s])
        assert np.linalg.norm(r) / np.linalg.norm(bs[s]) <= 1e-10
    assert np.all(xs[0].imag == 0.0)  # mean system stays real
    c.close()


def test_omega_zero_and_conjugate_on_device(F):
    m, Q, K = case()
    c = _ctx(F, m, Q)
    c.set_harmonics(np.array([[0.0], [18.0], [-18.0]]))
    b = synth.rhs(m.n_cells, 4)
    st, rep, xs = _solve(c, [0, 0, 0, 1, 2], [b, b.real, b.imag, b, np.conj(b)], kind="dilu", max_sweeps=30,
                         rtol=0.0)
    # omega = 0: complex RHS splits into two real mean solves
    assert relerr(xs[0], xs[1] + 1j * xs[2]) <= 1e-13
    # -omega with the conjugate RHS gives the conjugate iterate
    assert relerr(np.conj(xs[4]), xs[3]) <= 1e-13
    c.close()


def test_ragged_tiles_and_zero_rhs(F):
    m, Q, K = case(shape=(7, 5, 3), seed=3)  # 105 cells: ragged last tile of each colour
    c = _ctx(F, m, Q)
    om = np.array([[0.0], [25.0]])
    c.set_harmonics(om)
    col, nc = c.ordering()
    b1 = synth.rhs(m.n_cells, 1)
    st, rep, xs = _solve(c, [1, 1], [b1, np.zeros_like(b1)], kind="dilu", max_sweeps=40, rtol=0.0)
    x_or, _ = solve.richardson(K, m.volume, m.zone, om[1], b1, col, "DILU", rtol=0.0, max_sweeps=40)
    assert itererr(xs[0], x_or) <= ITER_TOL
    assert rep[1]["sweeps"] == 0 and np.all(xs[1] == 0) and rep[1]["status"] == 0
    # max_sweeps = 0 leaves x0 untouched
    x0 = synth.rhs(m.n_cells, 7)
    st, rep, xs = _solve(c, [1], [b1], x0s=[x0], kind="dilu", max_sweeps=0, rtol=1e-8)
    assert np.array_equal(xs[0], x0) and rep[0]["sweeps"] == 0
    c.close()


def test_nonzero_initial_guess(F):
    m, Q, K = case()
    c = _ctx(F, m, Q)
    om = synth.omegas_single_zone(1)
    c.set_harmonics(om)
    col, _ = c.ordering()
    b = synth.rhs(m.n_cells, 1)
    x0 = 0.1 * synth.rhs(m.n_cells, 9)
    st, rep, xs = _solve(c, [1], [b], x0s=[x0], kind="dilu", max_sweeps=17, rtol=0.0)
    x_or, _ = solve.richardson(K, m.volume, m.zone, om[1], b, col, "DILU", x0=x0, rtol=0.0, max_sweeps=17)
    assert itererr(xs[0], x_or) <= ITER_TOL
    c.close()


@pytest.mark.parametrize("hybrid", [0, 1])
def test_general_colouring_with_triangles(F, hybrid):
    """Three-row mesh with triangles (greedy colouring, 4 colours, the last two a small
    remainder): the general forward/backward passes (hybrid 0) and the two-colour passes
    plus remainder passes (hybrid 1, the default here) both give the oracle's DILU / SGS
    iterates on that colouring and converge to the dense solution."""
    m = synth.multi_row(6, 8, 4, n_blades=(36, 60, 48), seed=5)
    Q = synth.flow_state(m, 5)
    K = assemble.assemble(m, Q)
    c = _ctx(F, m, Q)
    c.tune(hybrid=hybrid)
    col, nc = c.ordering()
    assert nc >= 3 and ordering.is_valid(col, m.edges)
    om = synth.omegas_multi_row(2, (36, 60, 48))
    c.set_harmonics(om)
    bs = [synth.rhs(m.n_cells, s, real=(s == 0)) for s in range(3)]
    for kind in ("dilu", "sgs"):
        st, rep, xs = _solve(c, [0, 1, 2], bs, kind=kind, max_sweeps=25, rtol=0.0)
        for s in range(3):
            x_or, _ = solve.richardson(K, m.volume, m.zone, om[s], bs[s], col, kind.upper(), rtol=0.0,
                                       max_sweeps=25)
            assert itererr(xs[s], x_or) <= ITER_TOL, (kind, s)
    st, rep, xs = _solve(c, [0, 1, 2], bs, kind="dilu", max_sweeps=2000, rtol=1e-11)
    for s in range(3):
        xd = solve.dense_solve(K, m.volume, m.zone, om[s], bs[s])
        assert relerr(xs[s], xd) <= 1e-9
    c.close()


def test_chain_natural_order_exact(F):
    m = synth.chain(12)
    Q = synth.flow_state(m, 3)
    K = assemble.assemble(m, Q)
    nat = ordering.natural_colouring(m.n_cells)
    c = _ctx(F, m, Q, ordering_="user", user_colour=nat)
    c.set_harmonics(np.array([[18.0]]))
    b = synth.rhs(m.n_cells, 1)
    st, rep, xs = _solve(c, [0], [b], kind="dilu", max_sweeps=1, rtol=0.0)
    xd = solve.dense_solve(K, m.volume, m.zone, np.array([18.0]), b)
    assert relerr(xs[0], xd) <= 1e-12
    c.close()


def test_set_blocks_random_matrix(F):
    # raw blocks (any matrix on the pattern): a perturbed Jacobian with a random scaling
    m, Q, K = case(shape=(9, 6, 5), seed=8)
    rng = np.random.default_rng(0)
    K2 = K.copy()
    K2.offd = K.offd * (1.0 + 0.2 * rng.standard_normal(K.offd.shape))
    K2.diag = K.diag * 1.2 + 0.01 * np.abs(K.diag).max() * rng.standard_normal(K.diag.shape)
    import torch
    c = F.Context(m)
    d, o = blocks_user_layout(K2)
    c.set_blocks(to_dev(d), to_dev(o))
    om = np.array([[0.0], [30.0]])
    c.set_harmonics(om)
    col, _ = c.ordering()
    bs = [synth.rhs(m.n_cells, 0, real=True), synth.rhs(m.n_cells, 1)]
    st, rep, xs = _solve(c, [0, 1], bs, kind="dilu", max_sweeps=20, rtol=0.0)
    for s in range(2):
        x_or, _ = solve.richardson(K2, m.volume, m.zone, om[s], bs[s], col, "DILU", rtol=0.0, max_sweeps=20)
        assert itererr(xs[s], x_or) <= ITER_TOL
    c.close()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_reduced_precision_defect_correction(F, storage):
    """FP32 / BF16 blocks, FP32 sweeps, FP64 outer residual from the FP64 state: the
    iteration reaches the FP64 solution (rel. residual <= 1e-10 of the exact operator);
    OUTER_STORED converges to the rounded system instead."""
    m, Q, K = case()
    om = synth.omegas_single_zone(1)
    bs = [synth.rhs(m.n_cells, 0, real=True), synth.rhs(m.n_cells, 1)]
    c = _ctx(F, m, Q, storage=storage, outer="exact")
    c.set_harmonics(om)
    st, rep, xs = _solve(c, [0, 1], bs, kind="dilu", max_sweeps=3000, rtol=1e-10)
    assert st == 0
    for s in range(2):
        xd = solve.dense_solve(K, m.volume, m.zone, om[s], bs[s])
        r = bs[s] - solve.apply(K, solve.system_diag(K, m.volume, m.zone, om[s]), xs[s])
        assert np.linalg.norm(r) / np.linalg.norm(bs[s]) <= 1.5e-10
        assert relerr(xs[s], xd) <= 1e-8
        assert rep[s]["outer"] >= 1
    c.close()
    c = _ctx(F, m, Q, storage=storage, outer="stored")
    c.set_harmonics(om)
    st, rep, xs = _solve(c, [0, 1], bs, kind="dilu", max_sweeps=3000, rtol=1e-11)
    Kr = rounded(K, storage)
    for s in range(2):
        xr = solve.dense_solve(Kr, m.volume, m.zone, om[s], bs[s])
        xd = solve.dense_solve(K, m.volume, m.zone, om[s], bs[s])
        assert relerr(xs[s], xr) <= 1e-8
        # the rounded system's solution differs from the FP64 one by the storage error
        assert relerr(xr, xd) > 1e-12
    c.close()


def _raw_nondominant(K, seed=3):
    """Raw blocks far from the assembled Rusanov form: diagonal blocks with two row pairs
    swapped plus noise (not diagonally dominant, so the first-colour solve pivots and
    the factor inverses are full, unscaled matrices) and couplings perturbed by 20 %."""
    rng = np.random.default_rng(seed)
    K2 = K.copy()
    perm = np.array([1, 0, 2, 3, 5, 4])
    K2.diag = K.diag[:, perm, :] + 0.05 * np.abs(K.diag).max() * rng.standard_normal(K.diag.shape)
    K2.offd = K.offd * (1.0 + 0.2 * rng.standard_normal(K.offd.shape))
    return K2


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("mesh", ["hex", "three_row"])
def test_reduced_precision_raw_blocks(F, storage, mesh):
    """FP32 / BF16 storage on raw, non-dominant blocks: the FP16 factor inverses (with
    their power-of-two row scale) and the pivoting first-colour solve precondition the
    FP32 sweeps, and the FP64 defect correction with the FP64 shadow of the raw blocks
    still reaches the FP64 solution, in about the FP64 iteration's sweep count."""
    if mesh == "hex":
        m, Q, K = case(shape=(9, 6, 5), seed=8)
        om = np.array([[0.0], [30.0]])
    else:
        m = synth.multi_row(4, 4, 3, n_blades=(36, 60, 48), seed=5)
        K = assemble.assemble(m, synth.flow_state(m, 5))
        om = synth.omegas_multi_row(1, (36, 60, 48))
    K2 = _raw_nondominant(K)
    bs = [synth.rhs(m.n_cells, 0, real=True), synth.rhs(m.n_cells, 1)]
    for kind in ("dilu", "sgs"):
        c = F.Context(m, storage=storage, outer="exact")
        d, o = blocks_user_layout(K2)
        c.set_blocks(to_dev(d), to_dev(o))
        c.set_harmonics(om)
        col, nc = c.ordering()
        assert (nc == 2) == (mesh == "hex")
        st, rep, xs = _solve(c, [0, 1], bs, kind=kind, max_sweeps=4000, rtol=1e-10)
        assert st == 0, rep
        for s in range(2):
            Ds = solve.system_diag(K2, m.volume, m.zone, om[s])
            r = bs[s] - solve.apply(K2, Ds, xs[s])
            assert np.linalg.norm(r) / np.linalg.norm(bs[s]) <= 1.5e-10, (kind, s)
            assert relerr(xs[s], solve.dense_solve(K2, m.volume, m.zone, om[s], bs[s])) <= 1e-8, (kind, s)
            _, info = solve.richardson(K2, m.volume, m.zone, om[s], bs[s], col, kind.upper(), rtol=1e-10,
                                       max_sweeps=4000)
            assert rep[s]["sweeps"] <= 1.5 * info.sweeps + 16, (kind, s, rep[s]["sweeps"], info.sweeps)
        c.close()


def test_deterministic_bitwise(F):
    m, Q, K = case()
    c = _ctx(F, m, Q)
    c.set_harmonics(synth.omegas_single_zone(1))
    bs = [synth.rhs(m.n_cells, 0, real=True), synth.rhs(m.n_cells, 1)]
    _, r1, x1 = _solve(c, [0, 1], bs, kind="dilu", max_sweeps=200, rtol=1e-9)
    _, r2, x2 = _solve(c, [0, 1], bs, kind="dilu", max_sweeps=200, rtol=1e-9)
    for a, b in zip(x1, x2):
        assert np.array_equal(a, b)
    assert [r["sweeps"] for r in r1] == [r["sweeps"] for r in r2]
    c.close()


def test_residual_entry_point(F):
    m, Q, K = case()
    c = _ctx(F, m, Q)
    om = synth.omegas_single_zone(1)
    c.set_harmonics(om)
    import torch
    x = synth.rhs(m.n_cells, 3)
    b = synth.rhs(m.n_cells, 4)
    r = torch.empty((m.n_cells, 6), dtype=torch.complex128, device="cuda")
    n2 = c.residual(1, to_dev(x), to_dev(b), r)
    rr = b - solve.apply(K, solve.system_diag(K, m.volume, m.zone, om[1]), x)
    assert relerr(r.cpu().numpy(), rr) <= 1e-13
    assert abs(n2 - np.linalg.norm(rr) ** 2) <= 1e-12 * n2
    c.close()


def test_explicit_scheme_is_block_jacobi(F):
    m, Q, K = case()
    Ke = assemble.assemble(m, Q, scheme="explicit")
    c = _ctx(F, m, Q, scheme="explicit")
    om = np.array([[18.0]])
    c.set_harmonics(om)
    b = synth.rhs(m.n_cells, 1)
    st, rep, xs = _solve(c, [0], [b], kind="jacobi", max_sweeps=1, rtol=0.0)
    xd = solve.dense_solve(Ke, m.volume, m.zone, om[0], b)
    assert relerr(xs[0], xd) <= 1e-13
    c.close()


def test_factor_slot_pool(F):
    # fewer factor slots than systems: systems are factored batch by batch into the pool
    m, Q, K = case()
    c = _ctx(F, m, Q, factor_slots=1)
    om = synth.omegas_single_zone(3)
    c.set_harmonics(om)
    col, _ = c.ordering()
    bs = [synth.rhs(m.n_cells, s, real=(s == 0)) for s in range(4)]
    st, rep, xs = _solve(c, [0, 1, 2, 3], bs, kind="dilu", max_sweeps=10, rtol=0.0)
    for s in range(4):
        x_or, _ = solve.richardson(K, m.volume, m.zone, om[s], bs[s], col, "DILU", rtol=0.0, max_sweeps=10)
        assert itererr(xs[s], x_or) <= ITER_TOL
    mem1 = c.memory()
    c.close()
    c = _ctx(F, m, Q, factor_slots=1)
    c.set_harmonics(synth.omegas_single_zone(10))
    _solve(c, list(range(11)), [synth.rhs(m.n_cells, s) for s in range(11)], kind="dilu", max_sweeps=2, rtol=0.0)
    mem2 = c.memory()
    assert mem2["matrix_bytes"] == mem1["matrix_bytes"]
    assert mem2["factor_bytes"] == mem1["factor_bytes"]
    c.close()


def test_graph_replay_bitwise_matches_direct(F):
    # the sweep loop replayed from a captured graph gives the same bits as direct
    # launches, solve after solve (eager work in between)
    m, Q, K = case(shape=(12, 9, 7), seed=6)
    c = _ctx(F, m, Q)
    c.set_harmonics(synth.omegas_single_zone(3))
    bs = [synth.rhs(m.n_cells, s, real=(s == 0)) for s in range(4)]
    _, r0, x0 = _solve(c, [0, 1, 2, 3], bs, kind="dilu", max_sweeps=300, rtol=1e-9, check_every=8)
    for rep in range(3):
        _, r1, x1 = _solve(c, [0, 1, 2, 3], bs, kind="dilu", max_sweeps=300, rtol=1e-9, check_every=8,
                           use_graph=True)
        for a, b in zip(x0, x1):
            assert np.array_equal(a, b), rep
        assert [r["sweeps"] for r in r0] == [r["sweeps"] for r in r1]
        c.residual(1, to_dev(x1[1]), to_dev(bs[1]))  # eager work between replays
    # reduced precision with graphs
    c2 = _ctx(F, m, Q, storage="f32")
    c2.set_harmonics(synth.omegas_single_zone(3))
    _, s0, y0 = _solve(c2, [0, 1, 2, 3], bs, kind="dilu", max_sweeps=500, rtol=1e-9)
    _, s1, y1 = _solve(c2, [0, 1, 2, 3], bs, kind="dilu", max_sweeps=500, rtol=1e-9, use_graph=True)
    for a, b in zip(y0, y1):
        assert np.array_equal(a, b)
    c.close()
    c2.close()


def test_first_colour_solve_without_pivoting(F):
    # assembled Rusanov diagonals are dominant (pivot-free solve); raw blocks with a
    # non-dominant diagonal take the pivoting solve; both match the oracle
    m, Q, K = case(shape=(9, 6, 5), seed=8)
    rng = np.random.default_rng(3)
    K2 = K.copy()
    perm = np.array([1, 0, 2, 3, 5, 4])
    K2.diag = K.diag[:, perm, :] + 0.05 * np.abs(K.diag).max() * rng.standard_normal(K.diag.shape)
    om = np.array([[0.0], [30.0]])
    bs = [synth.rhs(m.n_cells, 0, real=True), synth.rhs(m.n_cells, 1)]
    for KK in (K, K2):
        c = F.Context(m)
        d, o = blocks_user_layout(KK)
        c.set_blocks(to_dev(d), to_dev(o))
        c.set_harmonics(om)
        col, _ = c.ordering()
        st, rep, xs = _solve(c, [0, 1], bs, kind="sgs", max_sweeps=12, rtol=0.0)
        for s in range(2):
            x_or, _ = solve.richardson(KK, m.volume, m.zone, om[s], bs[s], col, "SGS", rtol=0.0, max_sweeps=12)
            assert itererr(xs[s], x_or) <= ITER_TOL
        c.close()


def test_every_kernel_shape_covers_all_systems(F):
    # 9 systems: every (lanes per row, systems per lane) request must still sweep all
    # of them, and the per-system arithmetic does not depend on the shape
    m, Q, K = case(shape=(10, 7, 5), seed=12)
    om = synth.omegas_single_zone(8)
    bs = [synth.rhs(m.n_cells, s, real=(s == 0)) for s in range(9)]
    ref = None
    for lpr in (0, 1, 2, 4):
        for spw in (0, 1, 2, 4):
            c = _ctx(F, m, Q)
            c.set_harmonics(om)
            c.tune(spw, lpr)
            st, rep, xs = _solve(c, list(range(9)), bs, kind="dilu", max_sweeps=15, rtol=0.0)
            assert all(r["sweeps"] == 15 for r in rep), (lpr, spw)
            if ref is None:
                ref = xs
                col, _ = c.ordering()
                for s in (0, 4, 8):
                    x_or, _ = solve.richardson(K, m.volume, m.zone, om[s], bs[s], col, "DILU", rtol=0.0,
                                               max_sweeps=15)
                    assert itererr(xs[s], x_or) <= ITER_TOL
            else:
                for a, b in zip(ref, xs):
                    assert np.array_equal(a, b), (lpr, spw)
            c.close()


def test_graph_replay_after_buffer_reallocation(F):
    """Captured sweep graphs hold device addresses (factor slots, the omega table,
    partial sums).  Changing the system count reallocates those; replays must never use
    a freed buffer.  Memory released in between is refilled with NaN by fresh
    allocations, so a stale address would show up as a non-finite or wrong result."""
    import torch
    m, Q, K = case()
    om = synth.omegas_single_zone(3, 36)
    c = _ctx(F, m, Q)
    junk = []
    for k in (1, 3, 2, 4, 4):
        c.set_harmonics(om[:k])
        bs = [synth.rhs(m.n_cells, s) for s in range(k)]
        _, _, xg = _solve(c, list(range(k)), bs, max_sweeps=40, rtol=0.0, use_graph=True, check_every=4)
        junk += [torch.full((1 << 20,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(4)]
        _, _, xd = _solve(c, list(range(k)), bs, max_sweeps=40, rtol=0.0, use_graph=False, check_every=4)
        for a, b in zip(xg, xd):
            assert np.all(np.isfinite(a))
            assert np.array_equal(a, b)
    c.close()


@pytest.mark.parametrize("hybrid", [0, 2])
def test_every_general_path_shape_covers_all_systems(F, hybrid):
    # general colouring (triangles): 11 systems under every kernel shape, iterates equal
    # the oracle's and do not depend on the shape, for the general passes and for the
    # two-colour plus remainder passes
    m = synth.multi_row(5, 6, 3, n_blades=(36, 60, 48), seed=7)
    Q = synth.flow_state(m, 7)
    K = assemble.assemble(m, Q)
    om = synth.omegas_multi_row(10, (36, 60, 48))
    bs = [synth.rhs(m.n_cells, s, real=(s == 0)) for s in range(11)]
    ref = None
    for lpr in (0, 1, 2, 4):
        for spw in (0, 1, 4):
            c = _ctx(F, m, Q)
            c.set_harmonics(om)
            c.tune(spw, lpr, hybrid=hybrid)
            st, rep, xs = _solve(c, list(range(11)), bs, kind="dilu", max_sweeps=12, rtol=0.0)
            assert all(r["sweeps"] == 12 for r in rep), (lpr, spw)
            if ref is None:
                ref = xs
                col, nc = c.ordering()
                assert nc >= 3
                for s in (0, 5, 10):
                    x_or, _ = solve.richardson(K, m.volume, m.zone, om[s], bs[s], col, "DILU", rtol=0.0,
                                               max_sweeps=12)
                    assert itererr(xs[s], x_or) <= ITER_TOL
            else:
                for a, b in zip(ref, xs):
                    assert np.array_equal(a, b), (lpr, spw)
            c.close()


@pytest.mark.parametrize("n_sys", [2, 4, 7])
def test_wave_groups_bitwise(F, n_sys):
    """One wave per workgroup (FNLH_TUNE_WAVE_GROUPS) changes only the dispatch of the
    two-colour passes: the iterates are bitwise those of a tile per workgroup."""
    m, Q, K = case(shape=(10, 7, 5), seed=13)
    om = synth.omegas_single_zone(n_sys - 1)
    bs = [synth.rhs(m.n_cells, s, real=(s == 0)) for s in range(n_sys)]
    out = []
    for wg in (0, 1):
        c = _ctx(F, m, Q)
        c.set_harmonics(om)
        c.tune(0, 0, wave_groups=wg)
        st, rep, xs = _solve(c, list(range(n_sys)), bs, kind="dilu", max_sweeps=15, rtol=0.0)
        out.append(xs)
        c.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("mesh,hybrid", [("hex", 1), ("three_row", 1), ("three_row", 0)])
def test_reduced_precision_three_systems_a_lane(F, storage, mesh, hybrid):
    """Eleven systems in one call (four lanes a row, three systems a lane: the passes that
    request every system's loads together and the next system's FP16 factor ahead) give
    each system the iterates it gets when swept alone (one system a lane), to FP32
    rounding; on the two-colour passes, the two-colour plus remainder passes and the
    general passes."""
    n = 11
    if mesh == "hex":
        m, Q, K = case(shape=(9, 6, 5), seed=8)
        om = synth.omegas_single_zone(n - 1)
    else:
        m = synth.multi_row(4, 4, 3, n_blades=(36, 60, 48), seed=5)
        Q = synth.flow_state(m, 5)
        om = synth.omegas_multi_row(n - 1, (36, 60, 48))
    bs = [synth.rhs(m.n_cells, s, real=(s == 0)) for s in range(n)]
    c = _ctx(F, m, Q, storage=storage)
    c.set_harmonics(om)
    c.tune(hybrid=hybrid)
    st, rep, xs = _solve(c, list(range(n)), bs, kind="dilu", max_sweeps=12, rtol=0.0)
    assert all(r["sweeps"] == 12 for r in rep)
    for s in (0, 3, 7, 10):
        _, rep1, x1 = _solve(c, [s], [bs[s]], kind="dilu", max_sweeps=12, rtol=0.0)
        assert rep1[0]["sweeps"] == 12
        assert relerr(xs[s], x1[0]) <= 1e-5, (s, relerr(xs[s], x1[0]))
    c.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_hybrid_matches_general_passes(F, storage):
    """The two-colour plus remainder sweep computes the general passes' DILU step: on a
    colouring with five colours (three past the second) the iterates agree to rounding
    after every sweep count, the stop test sees the same residual norms (same sweep
    counts to a 1e-10 drop) and both reach the dense solution; SGS likewise."""
    m = synth.multi_row(4, 4, 3, n_blades=(36, 60, 48), seed=5)
    Q = synth.flow_state(m, 5)
    K = assemble.assemble(m, Q)
    om = synth.omegas_multi_row(3, (36, 60, 48))
    bs = [synth.rhs(m.n_cells, s, real=(s == 0)) for s in range(4)]
    out = {}
    for hybrid in (0, 2):
        c = _ctx(F, m, Q, storage=storage)
        c.set_harmonics(om)
        c.tune(hybrid=hybrid)
        assert c.ordering()[1] == 5
        res = {}
        for kind in ("dilu", "sgs"):
            res[kind, 7] = _solve(c, list(range(4)), bs, kind=kind, max_sweeps=7, rtol=0.0)
            res[kind, "conv"] = _solve(c, list(range(4)), bs, kind=kind, max_sweeps=4000, rtol=1e-10)
        out[hybrid] = res
        c.close()
    tol = 1e-11 if storage == "f64" else 1e-4
    for kind in ("dilu", "sgs"):
        for s in range(4):
            assert itererr(out[2][kind, 7][2][s], out[0][kind, 7][2][s]) <= tol, (kind, s)
            xd = solve.dense_solve(K, m.volume, m.zone, om[s], bs[s])
            assert relerr(out[2][kind, "conv"][2][s], xd) <= 1e-8, (kind, s)
            assert out[2][kind, "conv"][0] == 0
        if storage == "f64":
            assert [r["sweeps"] for r in out[2][kind, "conv"][1]] == [r["sweeps"] for r in out[0][kind, "conv"][1]]


@pytest.mark.parametrize("mesh,hybrid", [("hex", 1), ("three_row", 1), ("three_row", 0)])
def test_residual_history_matches_oracle(F, mesh, hybrid):
    """fnlh_relax's residual history (FP64 blocks): entry m is ||b - K_s x^m|| after m
    sweeps as the stop test measured it, entry `sweeps` the returned x's; it equals the
    oracle's Richardson history sweep for sweep, on the two-colour, the two-colour plus
    remainder and the general passes."""
    if mesh == "hex":
        m, Q, K = case(shape=(9, 6, 5), seed=8)
        om = synth.omegas_single_zone(2)
    else:
        m = synth.multi_row(6, 8, 4, n_blades=(36, 60, 48), seed=5)
        Q = synth.flow_state(m, 5)
        K = assemble.assemble(m, Q)
        om = synth.omegas_multi_row(2, (36, 60, 48))
    c = _ctx(F, m, Q)
    c.tune(hybrid=hybrid)
    c.set_harmonics(om)
    col, _ = c.ordering()
    bs = [synth.rhs(m.n_cells, s, real=(s == 0)) for s in range(3)]
    xs = [to_dev(np.zeros((m.n_cells, 6), complex)) for _ in bs]
    st, rep, hist = c.relax([0, 1, 2], xs, [to_dev(b) for b in bs], kind="dilu", max_sweeps=3000, rtol=1e-9,
                            history=True)
    assert st == 0
    for s in range(3):
        n = rep[s]["sweeps"]
        assert len(hist[s]) == n + 1 and np.all(np.isfinite(hist[s]))
        _, info = solve.richardson(K, m.volume, m.zone, om[s], bs[s], col, "DILU", rtol=0.0, max_sweeps=n)
        # relative 1e-9, and near the tolerance the FP64 rounding of the residual itself
        # (about 1e-17 of the initial norm here) decides: 1e-14 of the initial norm
        np.testing.assert_allclose(hist[s], info.history, rtol=1e-9, atol=1e-14 * info.history[0])
        # the stop test: x^(n-1) is the first iterate at the tolerance, x^n is returned
        assert hist[s][-2] <= 1e-9 * hist[s][0] < hist[s][-3]
    c.close()


def test_residual_history_reduced_precision(F):
    """FP32 blocks: the history holds the initial FP64 residual, the inner iteration's
    residuals in between and the FP64 residual after each correction; it falls to the
    tolerance and ends at the returned x's residual."""
    m, Q, K = case()
    om = synth.omegas_single_zone(1)
    c = _ctx(F, m, Q, storage="f32")
    c.set_harmonics(om)
    bs = [synth.rhs(m.n_cells, s, real=(s == 0)) for s in range(2)]
    xs = [to_dev(np.zeros((m.n_cells, 6), complex)) for _ in bs]
    st, rep, hist = c.relax([0, 1], xs, [to_dev(b) for b in bs], kind="dilu", max_sweeps=3000, rtol=1e-10,
                            history=True)
    assert st == 0
    for s in range(2):
        h = hist[s]
        assert len(h) == rep[s]["sweeps"] + 1 and np.all(np.isfinite(h)) and np.all(h > 0)
        assert abs(h[0] - np.linalg.norm(bs[s])) <= 1e-12 * h[0]
        assert abs(h[-1] - rep[s]["rel_res"] * rep[s]["res0"]) <= 1e-12 * h[0]
        assert h[-1] <= 1e-10 * h[0] and h[len(h) // 2] < 1e-3 * h[0]
    c.close()
