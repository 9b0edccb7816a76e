"""fnlh_residual_noalloc against fnlh_residual, through the C ABI: the same kernels on the
library's device scratch array instead of context buffers, so r and ||r||^2 must agree
bitwise.  Two calls in a row share the array, the second on a smaller mesh (the first
call's contents are left behind and must not leak into it); a mesh too large for the
array is refused with an error."""
import numpy as np
import pytest

from paper_2404_01407_amd import synth

from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2404_01407_amd import fnlh
    return fnlh


def _ctx(F, shape, storage, seed):
    m = synth.passage_block(*shape, 36, seed=seed)
    c = F.Context(m, storage=storage)
    c.assemble_jacobian(to_dev(synth.flow_state(m, seed)), eps=0.6, sigma=50.0)
    c.set_harmonics(synth.omegas_single_zone(2, 36))
    return m, c


def _check(F, c, m, sys, seed):
    import torch
    rng = np.random.default_rng(seed)
    x = to_dev(rng.standard_normal((m.n_cells, 6)) + 1j * rng.standard_normal((m.n_cells, 6)))
    b = to_dev(synth.rhs(m.n_cells, sys, real=(sys == 0)))
    r_ref = torch.empty_like(x)
    n2_ref = c.residual(sys, x, b, r_ref)
    r = torch.full_like(x, complex(np.nan, np.nan))
    n2 = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    c.residual_noalloc(sys, x, b, r, n2)
    n2_only = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    c.residual_noalloc(sys, x, b, None, n2_only)       # norm only: two staging vectors
    torch.cuda.synchronize()
    assert torch.equal(r, r_ref)
    assert float(n2.item()) == n2_ref and float(n2_only.item()) == n2_ref
    assert np.isfinite(n2_ref) and n2_ref > 0


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_noalloc_residual_equals_residual_two_calls(F, storage):
    big_m, big = _ctx(F, (40, 30, 30), storage, 41)        # 36,000 cells, ragged last tiles
    small_m, small = _ctx(F, (10, 7, 5), storage, 42)      # 350 cells, after the big call
    _check(F, big, big_m, 1, 1)
    _check(F, small, small_m, 2, 2)
    _check(F, big, big_m, 0, 3)                             # and back to the larger one
    big.close()
    small.close()


def test_noalloc_residual_frozen_system(F):
    m, c = _ctx(F, (12, 6, 5), "f64", 43)
    c.set_frozen_turbulence([0, 1, 0])
    _check(F, c, m, 1, 4)
    c.close()


def test_noalloc_residual_refuses_a_mesh_beyond_the_scratch(F):
    import torch
    assert F.LIB.fnlh_noalloc_scratch_bytes() == 64 << 20
    m, c = _ctx(F, (80, 50, 60), "f32", 44)                # 240,000 cells: three vectors exceed 64 MiB
    x = torch.zeros((m.n_cells, 6), dtype=torch.complex128, device="cuda")
    with pytest.raises(F.FnlhError, match="scratch"):
        c.residual_noalloc(0, x, x, torch.empty_like(x))
    c.close()
