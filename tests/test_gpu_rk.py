"""GPU parity of the RK(5,3) pseudo-time driver (fnlh_rusanov_residual, fnlh_rk_mean,
fnlh_rk_harmonic) against the oracle's driver: the Rusanov residual element by element,
whole pseudo-time steps of the mean flow and of a harmonic with fixed sweep counts in
FP64 (iterates to 1e-10: the nonlinear stages amplify rounding only mildly over a few
steps), and the harmonic fixed point against the dense linearised solution."""
import numpy as np
import pytest

from oracle import assemble, rk, solve
from paper_2404_01407_amd import synth

from gpu_helpers import relerr, to_dev

pytestmark = pytest.mark.gpu

STEP_TOL = 1e-10


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2404_01407_amd import fnlh
    return fnlh


def _mesh(kind, seed=5):
    if kind == "passage":
        m = synth.passage_block(12, 6, 4, 36, seed=seed)           # 288 cells, several tiles
    else:
        m = synth.cascade_block(8, 5, 3, 36, seed=seed)            # odd pitch: general colouring
    return m, synth.flow_state(m, seed)


def _far_field(m, Q, seed=3):
    rng = np.random.default_rng(seed)
    return Q[m.bface_cell] * (1.0 + 0.05 * rng.standard_normal((m.bface_cell.size, 6)))


@pytest.mark.parametrize("kind", ["passage", "cascade"])
@pytest.mark.parametrize("with_ff", [False, True])
def test_rusanov_residual_matches_oracle(F, kind, with_ff):
    m, Q = _mesh(kind)
    Qff = _far_field(m, Q) if with_ff else None
    c = F.Context(m)
    R, n2 = c.rusanov_residual(to_dev(Q), None if Qff is None else to_dev(Qff))
    R_or = rk.nonlinear_residual(m, Q, Qff)
    assert relerr(R.cpu().numpy(), R_or) <= 1e-13
    assert abs(n2 - np.sum(R_or ** 2)) <= 1e-12 * np.sum(R_or ** 2)
    c.close()


@pytest.mark.parametrize("kind", ["passage", "cascade"])
@pytest.mark.parametrize("scheme,sigma", [("implicit", 50.0), ("explicit", 1.0)])
def test_rk_mean_steps_match_oracle(F, kind, scheme, sigma):
    import torch
    m, Q = _mesh(kind)
    Qff = _far_field(m, Q)
    c = F.Context(m)
    st = to_dev(Q)
    c.assemble_jacobian(st, to_dev(Qff), eps=0.6, sigma=sigma, scheme=scheme)
    c.set_harmonics(np.zeros((1, m.n_zones)))
    col, _ = c.ordering()
    n_steps = 3
    status, hist = c.rk_mean(0, st, n_steps, eps=0.6, sigma=sigma, scheme=scheme, bstate=to_dev(Qff),
                             max_sweeps=10, rtol=0.0)
    torch.cuda.synchronize()
    assert status in (F.OK, F.NOT_CONVERGED)
    Qo = Q.copy()
    h_or = []
    for _ in range(n_steps):
        Qo, r0 = rk.mean_step(m, Qo, col, eps=0.6, sigma=sigma, scheme=scheme, rtol=0.0, max_sweeps=10, Qff=Qff)
        h_or.append(r0)
    assert relerr(st.cpu().numpy(), Qo) <= STEP_TOL
    np.testing.assert_allclose(hist, h_or, rtol=1e-11)
    assert relerr(Qo, Q) > 1e-6                                      # the steps did move the state
    c.close()


def test_rk_mean_uniform_state_is_steady(F):
    import torch
    m, _ = _mesh("passage")
    Q = np.tile(np.array([1.0, 0.5, 0.1, -0.2, 2.7, 1e-4]), (m.n_cells, 1))
    c = F.Context(m)
    st = to_dev(Q)
    c.assemble_jacobian(st)
    c.set_harmonics(np.zeros((1, m.n_zones)))
    _, hist = c.rk_mean(0, st, 2, max_sweeps=10, rtol=1e-2)
    torch.cuda.synchronize()
    assert np.all(hist <= 1e-13)
    np.testing.assert_allclose(st.cpu().numpy(), Q, rtol=0, atol=1e-13)
    c.close()


@pytest.mark.parametrize("kind", ["passage", "cascade"])
@pytest.mark.parametrize("scheme,sigma", [("implicit", 50.0), ("explicit", 1.0)])
def test_rk_harmonic_steps_match_oracle(F, kind, scheme, sigma):
    import torch
    m, Q = _mesh(kind)
    om = np.array([[0.0], [18.0]]) if m.n_zones == 1 else np.zeros((2, m.n_zones))
    om[1] = 18.0
    rng = np.random.default_rng(7)
    fh = rng.standard_normal((m.n_cells, 6)) + 1j * rng.standard_normal((m.n_cells, 6))
    c = F.Context(m)
    c.assemble_jacobian(to_dev(Q), eps=0.6, sigma=sigma, scheme=scheme)
    c.set_harmonics(om)
    col, _ = c.ordering()
    qh = to_dev(np.zeros_like(fh))
    n_steps = 3
    status, hist = c.rk_harmonic(1, qh, to_dev(fh), n_steps, max_sweeps=10, rtol=0.0)
    torch.cuda.synchronize()
    Qo = np.zeros_like(fh)
    h_or = []
    for _ in range(n_steps):
        Qo, r0 = rk.harmonic_step(m, Q, Qo, fh, om[1], col, eps=0.6, sigma=sigma, scheme=scheme, rtol=0.0,
                                  max_sweeps=10)
        h_or.append(r0)
    assert relerr(qh.cpu().numpy(), Qo) <= STEP_TOL
    np.testing.assert_allclose(hist, h_or, rtol=1e-11)
    c.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_rk_harmonic_reaches_linearised_solution(F, storage):
    """The fixed point is the solution of (J + i omega V) q = f whatever the stage solves'
    precision: FP32 blocks only change K, the preconditioner."""
    import torch
    m, Q = _mesh("passage")
    om = np.array([[0.0], [18.0]])
    rng = np.random.default_rng(1)
    fh = rng.standard_normal((m.n_cells, 6)) + 1j * rng.standard_normal((m.n_cells, 6))
    J = assemble.residual_jacobian(Q, m.edges, m.area, m.bface_cell, m.bface_area)
    x_star = solve.dense_solve(J, m.volume, m.zone, om[1], fh)
    c = F.Context(m, storage=storage)
    c.assemble_jacobian(to_dev(Q))
    c.set_harmonics(om)
    qh = to_dev(np.zeros_like(fh))
    _, hist = c.rk_harmonic(1, qh, to_dev(fh), 120, max_sweeps=10, rtol=1e-2)
    torch.cuda.synchronize()
    assert hist[-1] <= 1e-9 * hist[0], hist[-1] / hist[0]
    assert relerr(qh.cpu().numpy(), x_star) <= 1e-8
    c.close()


def test_rk_harmonic_phase_lagged_fixed_point(F):
    """With phase-lagged periodic couplings the fixed point is the phased linearised
    solution (the residual and the stage solves both carry the phase)."""
    import torch
    m, Q = _mesh("cascade", seed=11)
    om = np.zeros((2, m.n_zones))
    om[1] = 18.0
    sig = np.array([0.0, 0.9])
    rng = np.random.default_rng(2)
    fh = rng.standard_normal((m.n_cells, 6)) + 1j * rng.standard_normal((m.n_cells, 6))
    J = assemble.residual_jacobian(Q, m.edges, m.area, m.bface_cell, m.bface_area)
    x_star = solve.dense_solve(solve.phase_lagged(J, m.edge_phase, sig[1]), m.volume, m.zone, om[1], fh)
    c = F.Context(m)
    c.assemble_jacobian(to_dev(Q))
    c.set_harmonics(om)
    c.set_phase_lag(m.edge_phase, sig)
    qh = to_dev(np.zeros_like(fh))
    _, hist = c.rk_harmonic(1, qh, to_dev(fh), 150, max_sweeps=10, rtol=1e-2)
    torch.cuda.synchronize()
    assert relerr(qh.cpu().numpy(), x_star) <= 1e-8, hist[-1] / hist[0]
    c.close()


def test_rk_errors(F):
    m, Q = _mesh("passage")
    c = F.Context(m)
    qh = to_dev(np.zeros((m.n_cells, 6), complex))
    with pytest.raises(F.FnlhError):
        c.rk_harmonic(0, qh, qh, 1)                                   # nothing assembled
    st = to_dev(Q)
    c.assemble_jacobian(st)
    c.set_harmonics(np.array([[0.0], [18.0]]))
    with pytest.raises(F.FnlhError):
        c.rk_mean(1, st, 1)                                           # omega != 0
    with pytest.raises(F.FnlhError):
        c.rk_mean(0, st, 1, kind="learned")
    with pytest.raises(F.FnlhError):
        c.rk_harmonic(2, qh, qh, 1)                                   # no such system
    c.close()
