"""GPU checks of the learned preconditioner: the matrix-core tile routine, the network's
forward pass and loss gradient against the FP64 oracle, Adam, training on pairs the
plain solver generates, and fnlh_relax with learned corrections (convergence to the
same bar as the plain method, rejection of useless or non-finite corrections).

Tolerances.  The kernels hold weights and activations in BF16 (unit roundoff 2^-9 =
2e-3) and accumulate in FP32.  The oracle is evaluated with the same BF16-rounded
weights, so what remains is the rounding of the node and edge inputs and of the hidden
activations at five points along the network; with fan-ins of 60-128 those add up to
an expected relative error of a few 1e-3 in the output.  The tests allow 3e-2 for the
output and 6e-2 per weight matrix for the gradient (plus a cosine of at least 0.998):
an order of magnitude over the expected rounding, far below the O(1) error of any
indexing or layout mistake (a transposed operand, a dropped edge, a wrong sign)."""
import numpy as np
import pytest

from oracle import learned, precision, solve
from paper_2404_01407_amd import synth

from gpu_helpers import blocks_user_layout, case, relerr, rounded, to_dev

pytestmark = pytest.mark.gpu

FWD_TOL = 3e-2
GRAD_TOL = 6e-2


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2404_01407_amd import fnlh
    return fnlh


@pytest.fixture(scope="module")
def small():
    m, Q, K = case(shape=(10, 7, 5), seed=31)          # 350 cells: 6 tiles, ragged tail
    om = synth.omegas_single_zone(2, 36)               # mean + 2 harmonics
    return m, Q, K, om


def _ctx(F, m, K, om, storage="f64"):
    c = F.Context(m, storage=storage)
    d, o = blocks_user_layout(K)
    c.set_blocks(to_dev(d), to_dev(o))
    c.set_harmonics(om)
    return c


def _weights(seed):
    w = learned.init_weights(seed)
    w[-64 * 12:] *= 10.0          # full-scale decoder so every layer carries signal
    return w.astype(np.float32)


def _bf16(w):
    return precision.round_bf16(np.asarray(w, np.float64))


def _cvec(rng, n):
    return rng.standard_normal((n, 6)) + 1j * rng.standard_normal((n, 6))


def test_mfma_tile_product(F, small):
    m, Q, K, om = small
    c = _ctx(F, m, K, om)
    rng = np.random.default_rng(5)
    a = rng.standard_normal((64, 64)).astype(np.float32)
    b = rng.standard_normal((64, 64)).astype(np.float32)
    bits = lambda x: (np.ascontiguousarray(x, np.float32).view(np.uint32) >> 16).astype(np.uint16)  # truncation
    ab, bb = bits(a), bits(b.T)
    av = (ab.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    bv = (bb.astype(np.uint32) << 16).view(np.float32).astype(np.float64).T
    out = F.mfma_selftest(c, ab, bb)
    ref = av @ bv
    assert np.abs(out - ref).max() <= 1e-5 * np.abs(av).max() * np.abs(bv).max() * 64
    c.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_forward_matches_oracle(F, small, storage):
    import torch
    m, Q, K, om = small
    Kr = rounded(K, storage)
    c = _ctx(F, m, Kr if storage == "f64" else K, om, storage)
    net = F.Network(c)
    w = _weights(7)
    net.set_weights(w)
    rng = np.random.default_rng(11)
    for s in (0, 2):
        r = _cvec(rng, m.n_cells)
        dx = net.apply(s, to_dev(r)).cpu().numpy()
        Ds = solve.system_diag(Kr, m.volume, m.zone, om[s])
        ref = learned.apply(_bf16(w), Kr, Ds, r)
        assert relerr(dx, ref) <= FWD_TOL, (storage, s, relerr(dx, ref))
        # homogeneity holds exactly up to the input rounding
        dx2 = net.apply(s, to_dev(4.0 * r)).cpu().numpy()
        assert relerr(dx2, 4.0 * dx) <= 1e-6
    torch.cuda.synchronize()
    net.close()
    c.close()


def _check_gradient(F, m, K, om, groups, seed):
    """Loss and gradient of two pairs against the oracle's backward pass, with the
    backward kernels launched on `groups` workgroups (0: automatic)."""
    c = _ctx(F, m, K, om)
    net = F.Network(c)
    net.set_grad_groups(groups)
    w = _weights(8)
    net.set_weights(w)
    rng = np.random.default_rng(seed)
    systems = [0, 1]
    rs = [_cvec(rng, m.n_cells) for _ in systems]
    es = [_cvec(rng, m.n_cells) for _ in systems]
    loss, g = net.loss_grad(systems, [to_dev(r) for r in rs], [to_dev(e) for e in es])
    wb = _bf16(w)
    Lref, gref = 0.0, np.zeros(learned.n_params())
    for s, r, e in zip(systems, rs, es):
        Ds = solve.system_diag(K, m.volume, m.zone, om[s])
        u, gg, sigma = learned.features(K, Ds, r)
        L, gr = learned.loss_and_grad(wb, u, gg, K.rows, K.cols, m.n_cells, learned.c2r(e / sigma))
        Lref += L / len(systems)
        gref += gr / len(systems)
    assert abs(loss - Lref) <= FWD_TOL * abs(Lref)
    offs = np.cumsum([0] + [a * b for a, b in learned.SHAPES])
    for k in range(5):
        a, b = g[offs[k]:offs[k + 1]].astype(np.float64), gref[offs[k]:offs[k + 1]]
        assert relerr(a, b) <= GRAD_TOL, (groups, k, relerr(a, b))
        assert a @ b / (np.linalg.norm(a) * np.linalg.norm(b)) >= 0.998, (groups, k)
    net.close()
    c.close()
    return g


def test_gradient_matches_oracle(F, small):
    m, Q, K, om = small
    _check_gradient(F, m, K, om, 0, 12)


@pytest.mark.parametrize("groups", [1, 2, 4])
def test_gradient_several_tiles_per_workgroup(F, small, groups):
    """The backward kernels sum the partials of tiles g, g + G, ... per workgroup: with
    G = 1, 2 or 4 workgroups on the 6 tiles of the 350-cell mesh each sums 6, 3 or
    1-2 tiles (the path every 200k-cell training step takes, about six tiles each)."""
    m, Q, K, om = small
    _check_gradient(F, m, K, om, groups, 12)


def test_gradient_more_tiles_than_workgroups(F):
    """36,000 cells = 563 tiles on the automatic 512 workgroups: 51 of them sum two
    tiles, the rest one."""
    m, Q, K = case(shape=(40, 30, 30), seed=33)
    om = synth.omegas_single_zone(1, 36)
    _check_gradient(F, m, K, om, 0, 34)


def _pairs(F, c, net, systems, per_system, sweeps, seed):
    """Pairs from the plain solver: with b = 0 the iterate after m DILU sweeps from a
    random start is minus its own error, and its residual is -K x."""
    import torch
    rng = np.random.default_rng(seed)
    zero = to_dev(np.zeros((c.n, 6), complex))
    for s in systems:
        for k in range(per_system):
            x = to_dev(_cvec(rng, c.n))
            c.relax([s], [x], [zero], kind="dilu", max_sweeps=int(sweeps[k % len(sweeps)]), rtol=0.0)
            r = torch.empty_like(x)
            c.residual(s, x, zero, r)
            net.add_pairs([s], [r], [-x])
    torch.cuda.synchronize()


def test_adam_step_on_device(F, small):
    m, Q, K, om = small
    c = _ctx(F, m, K, om)
    net = F.Network(c)
    w = _weights(9)
    net.set_weights(w)
    rng = np.random.default_rng(13)
    # BF16-representable pair, so the stored BF16 copy equals the FP64 input
    r = _bf16(_cvec(rng, m.n_cells).view(np.float64)).view(complex)
    e = _bf16(_cvec(rng, m.n_cells).view(np.float64)).view(complex)
    net.add_pairs([1], [to_dev(r)], [to_dev(e)])
    loss0, g = net.loss_grad([1], [to_dev(r)], [to_dev(e)])
    lr = np.float32(1e-3)
    hist = net.train(1, batch=1, lr=float(lr), seed=3)
    assert abs(hist[0] - loss0) <= 1e-6 * loss0
    w1 = net.get_weights()
    m1 = np.float32(0.1) * g
    v1 = np.float32(0.001) * g * g
    ref = w - lr * (m1 / np.float32(1 - 0.9)) / (np.sqrt(v1 / np.float32(1 - 0.999)) + np.float32(1e-8))
    np.testing.assert_allclose(w1, ref, rtol=2e-6, atol=2e-7 * float(lr))
    net.close()
    c.close()


def test_training_lowers_loss(F, small):
    m, Q, K, om = small
    c = _ctx(F, m, K, om)
    net = F.Network(c)
    net.set_weights(learned.init_weights(10).astype(np.float32))
    _pairs(F, c, net, [0, 1, 2], 8, [2, 4, 8, 16], seed=14)
    assert net.n_pairs() == 24
    hist = net.train(150, batch=4, lr=2e-3, seed=1)
    assert np.all(np.isfinite(hist))
    assert hist[-20:].mean() < 0.8 * hist[:10].mean(), (hist[:10].mean(), hist[-20:].mean())
    assert np.all(np.isfinite(net.get_weights()))
    net.close()
    c.close()


def _dense_solutions(K, m, om, systems, bs):
    out = []
    for s, b in zip(systems, bs):
        A = solve.dense(K, m.volume, m.zone, om[s])
        out.append(np.linalg.solve(A, b.reshape(-1)).reshape(-1, 6))
    return out


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_learned_relax_converges(F, small, storage):
    import torch
    m, Q, K, om = small
    c = F.Context(m, storage=storage)
    c.assemble_jacobian(to_dev(Q), eps=0.6, sigma=50.0)
    c.set_harmonics(om)
    net = F.Network(c)
    net.set_weights(_weights(15))
    rng = np.random.default_rng(16)
    systems = [0, 1, 2]
    bs = [_cvec(rng, m.n_cells) for _ in systems]
    xs = [to_dev(np.zeros((m.n_cells, 6), complex)) for _ in systems]
    st, rep = c.relax(systems, xs, [to_dev(b) for b in bs], kind="learned", max_sweeps=600, rtol=1e-10,
                      learn_every=8, check_every=4)
    torch.cuda.synchronize()
    assert st in (F.OK, F.FELL_BACK), rep
    ref = _dense_solutions(K, m, om, systems, bs)
    for j, r in enumerate(rep):
        assert r["rel_res"] <= 1e-10
        assert r["learned"] + r["fallbacks"] >= 1, r
        assert relerr(xs[j].cpu().numpy(), ref[j]) <= 1e-9
    net.close()
    c.close()


def test_nonfinite_corrections_are_rejected(F, small):
    import torch
    m, Q, K, om = small
    c = _ctx(F, m, K, om)
    net = F.Network(c)
    net.set_weights(np.full(F.NN_PARAMS, 1e30, np.float32))    # activations overflow
    rng = np.random.default_rng(17)
    b = _cvec(rng, m.n_cells)
    x = to_dev(np.zeros((m.n_cells, 6), complex))
    st, rep = c.relax([1], [x], [to_dev(b)], kind="learned", max_sweeps=600, rtol=1e-10, learn_every=8)
    torch.cuda.synchronize()
    # three rejections in a row switch the network off for the rest of the call
    assert st == F.FELL_BACK and rep[0]["status"] == F.FELL_BACK
    assert rep[0]["learned"] == 0 and rep[0]["fallbacks"] == 3
    assert np.all(np.isfinite(x.cpu().numpy()))
    ref = _dense_solutions(K, m, om, [1], [b])[0]
    assert relerr(x.cpu().numpy(), ref) <= 1e-9
    # zero weights: dx = 0 gives no descent at all and is rejected as well
    net.set_weights(np.zeros(F.NN_PARAMS, np.float32))
    x = to_dev(np.zeros((m.n_cells, 6), complex))
    st, rep = c.relax([1], [x], [to_dev(b)], kind="learned", max_sweeps=600, rtol=1e-10, learn_every=8)
    assert st == F.FELL_BACK and rep[0]["learned"] == 0 and rep[0]["fallbacks"] == 3
    assert relerr(x.cpu().numpy(), ref) <= 1e-9
    net.close()
    c.close()


def test_learned_general_colouring(F):
    import torch
    m = synth.multi_row(6, 5, 3, n_blades=(36, 60, 48), seed=5)
    Q = synth.flow_state(m, 5)
    om = synth.omegas_multi_row(1, (36, 60, 48))
    c = F.Context(m, storage="f64")
    c.assemble_jacobian(to_dev(Q), eps=0.6, sigma=50.0)
    c.set_harmonics(om)
    assert c.ordering()[1] > 2
    net = F.Network(c)
    net.set_weights(_weights(18))
    rng = np.random.default_rng(19)
    b = _cvec(rng, m.n_cells)
    x = to_dev(np.zeros((m.n_cells, 6), complex))
    st, rep = c.relax([1], [x], [to_dev(b)], kind="learned", max_sweeps=800, rtol=1e-10, learn_every=8)
    torch.cuda.synchronize()
    assert st in (F.OK, F.FELL_BACK), rep
    r = to_dev(np.zeros((m.n_cells, 6), complex))
    n2 = c.residual(1, x, to_dev(b), r)
    assert np.sqrt(n2) <= 1e-10 * rep[0]["res0"] * 1.0001
    net.close()
    c.close()


def test_network_requires_weights_and_one_per_context(F, small):
    m, Q, K, om = small
    c = _ctx(F, m, K, om)
    net = F.Network(c)
    with pytest.raises(F.FnlhError):
        net.apply(0, to_dev(np.zeros((m.n_cells, 6), complex)))
    with pytest.raises(F.FnlhError):
        F.Network(c)
    with pytest.raises(F.FnlhError):
        c.relax([0], [to_dev(np.zeros((m.n_cells, 6), complex))], [to_dev(np.ones((m.n_cells, 6), complex))],
                kind="learned", max_sweeps=10)
    net.close()
    with pytest.raises(F.FnlhError):   # detached: relax has no network any more
        c.relax([0], [to_dev(np.zeros((m.n_cells, 6), complex))], [to_dev(np.ones((m.n_cells, 6), complex))],
                kind="learned", max_sweeps=10)
    c.close()


def _uniform_start(seed, start, n_values):
    """The library's documented generator of random starts, written out in numpy:
    x_v = 2 u - 1, u = (mix(key + v) >> 11) 2^-53, key = mix(seed + golden (start + 1))."""
    M = np.uint64(0xFFFFFFFFFFFFFFFF)

    def mix(z):
        z = np.asarray(z, np.uint64)
        with np.errstate(over="ignore"):
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))

    with np.errstate(over="ignore"):
        key = mix(np.uint64(seed) + np.uint64(0x9E3779B97F4A7C15) * np.uint64(start + 1)) & M
        v = key + np.arange(n_values, dtype=np.uint64)
    u = (mix(v) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return (2.0 * u - 1.0).view(complex).reshape(-1, 6)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_generate_equals_the_call_sequence(F, small, storage):
    """fnlh_nn_generate stores bitwise the pairs that the documented sequence of
    fnlh_relax, fnlh_residual and fnlh_nn_add_pairs calls stores, starting from the
    documented counter-based random starts."""
    import torch
    m, Q, K, om = small
    c = F.Context(m, storage=storage)
    c.assemble_jacobian(to_dev(Q), eps=0.6, sigma=50.0)
    c.set_harmonics(om)
    net = F.Network(c)
    systems, starts, snaps, every, seed = [0, 2, 1], 2, 3, 4, 12345
    net.generate(systems, starts, snaps, every, seed=seed)
    assert net.n_pairs() == len(systems) * starts * snaps
    c2 = F.Context(m, storage=storage)   # a second pool, filled by the call sequence
    c2.assemble_jacobian(to_dev(Q), eps=0.6, sigma=50.0)
    c2.set_harmonics(om)
    ref = F.Network(c2)
    zero = to_dev(np.zeros((m.n_cells, 6), complex))
    for k in range(starts):
        xs = [to_dev(_uniform_start(seed, j * starts + k, 12 * m.n_cells)) for j in range(len(systems))]
        for t in range(snaps):
            c2.relax(systems, xs, [zero] * len(systems), kind="dilu", max_sweeps=every, rtol=0.0, check_every=16,
                     use_graph=True)
            for j, sy in enumerate(systems):
                r = torch.empty_like(xs[j])
                c2.residual(sy, xs[j], zero, r)
                ref.add_pairs([sy], [r], [-xs[j]])
    torch.cuda.synchronize()
    assert ref.n_pairs() == net.n_pairs()
    for k in range(net.n_pairs()):
        s1, r1, e1 = net.get_pair(k)
        s2, r2, e2 = ref.get_pair(k)
        assert s1 == s2
        assert torch.equal(r1, r2) and torch.equal(e1, e2), k
    # the pairs are what they claim: r = -K_s x and e = -x (BF16-rounded) for the last
    # iterate x of the last system
    s1, r1, e1 = net.get_pair(net.n_pairs() - 1)
    x = xs[-1].cpu().numpy()
    assert s1 == systems[-1]
    Ds = solve.system_diag(K, m.volume, m.zone, om[s1])
    rr = -solve.apply(K, Ds, x)
    np.testing.assert_allclose(r1.cpu().numpy(), rr, rtol=0, atol=1e-2 * np.abs(rr).max())
    np.testing.assert_allclose(e1.cpu().numpy(), -x, rtol=0, atol=1e-2 * np.abs(x).max())
    ref.close()
    c2.close()
    net.close()
    c.close()


def test_save_load_resumes_training_bitwise(F, small, tmp_path):
    """A checkpoint holds the FP32 weights, Adam's moments and step count: training
    resumed from it equals the uninterrupted run bitwise (weights and losses), and the
    restored network's output is the saved one's."""
    m, Q, K, om = small
    path = str(tmp_path / "net.fnlhnn")
    nets, ctxs = [], []
    for _ in range(2):
        c = _ctx(F, m, K, om)
        net = F.Network(c)
        net.generate([0, 1, 2], 2, 2, 4, seed=3)
        ctxs.append(c)
        nets.append(net)
    a, b = nets
    a.set_weights(_weights(21))
    a.train(6, batch=2, lr=1e-3, seed=1)
    a.save(path)
    h_a = a.train(5, batch=2, lr=1e-3, seed=2)
    b.set_weights(np.zeros(F.NN_PARAMS, np.float32))
    b.load(path)
    h_b = b.train(5, batch=2, lr=1e-3, seed=2)
    assert np.array_equal(h_a, h_b)
    assert np.array_equal(a.get_weights(), b.get_weights())
    rng = np.random.default_rng(22)
    r = to_dev(_cvec(rng, m.n_cells))
    assert np.array_equal(a.apply(1, r).cpu().numpy(), b.apply(1, r).cpu().numpy())
    # a file that is not a checkpoint is refused and leaves the network as it was
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"FNLHNN01" + bytes(40))
    with pytest.raises(F.FnlhError):
        b.load(str(bad))
    with pytest.raises(F.FnlhError):
        b.load(str(tmp_path / "missing.bin"))
    assert np.array_equal(a.get_weights(), b.get_weights())
    for net, c in zip(nets, ctxs):
        net.close()
        c.close()


def test_copy_state_equals_checkpoint(F, small):
    """Training state copied device to device continues exactly as the original."""
    m, Q, K, om = small
    ctxs = [_ctx(F, m, K, om) for _ in range(2)]
    a, b = [F.Network(c) for c in ctxs]
    for n in (a, b):
        n.generate([0, 2], 2, 2, 4, seed=5)
    a.set_weights(_weights(23))
    a.train(4, batch=2, lr=1e-3, seed=1)
    b.copy_state_from(a)
    assert np.array_equal(a.train(3, batch=2, lr=1e-3, seed=2), b.train(3, batch=2, lr=1e-3, seed=2))
    assert np.array_equal(a.get_weights(), b.get_weights())
    for n, c in zip((a, b), ctxs):
        n.close()
        c.close()


def test_network_width_is_checked(F, small):
    m, Q, K, om = small
    c = _ctx(F, m, K, om)
    with pytest.raises(F.FnlhError):
        F.Network(c, hidden=32)
    net = F.Network(c, hidden=64)
    net.close()
    c.close()
