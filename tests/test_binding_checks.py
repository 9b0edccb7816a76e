"""The Python binding checks every device argument before its pointer crosses the C ABI:
dtype (complex128 vectors, float64 states and blocks), shape, contiguity, device kind
and device index.  A wrong tensor must raise in Python, before any library call: a
complex64 vector passed through as a raw pointer would make the kernels read and write
twice its bytes.  The library is replaced by a stub that fails on any use, so these
tests need no GPU."""
import numpy as np
import pytest
import torch

from paper_2404_01407_amd import fnlh

N, E, B = 10, 13, 4


class _NoLib:
    def __getattr__(self, name):
        raise AssertionError(f"library function {name} called before the argument check")


@pytest.fixture()
def ctx(monkeypatch):
    monkeypatch.setattr(fnlh, "LIB", _NoLib())
    c = object.__new__(fnlh.Context)
    c.n, c.E, c.B, c.n_zones, c.device, c.n_sys, c.storage = N, E, B, 1, 0, 2, "f64"
    c.h = None
    yield c


def _net(ctx):
    nn = object.__new__(fnlh.Network)
    nn.ctx, nn.h = ctx, None
    return nn


VEC = (N, 6)


def _bad_vectors():
    """(tensor, expected exception) that the checks must refuse."""
    return [
        (torch.zeros(VEC, dtype=torch.complex64), TypeError),           # half the bytes
        (torch.zeros(VEC, dtype=torch.float64), TypeError),             # real instead of complex
        (torch.zeros((N + 1, 6), dtype=torch.complex128), ValueError),  # wrong shape
        (torch.zeros((6, N), dtype=torch.complex128).t(), ValueError),  # not contiguous
        (torch.zeros(VEC, dtype=torch.complex128), TypeError),          # host memory
        (np.zeros(VEC, complex), TypeError),                            # not a tensor
    ]


def _bad_states():
    return [
        (torch.zeros(VEC, dtype=torch.float32), TypeError),
        (torch.zeros(VEC, dtype=torch.complex128), TypeError),
        (torch.zeros((N, 5), dtype=torch.float64), ValueError),
        (torch.zeros(VEC, dtype=torch.float64), TypeError),             # host memory
    ]


@pytest.mark.parametrize("k", range(6))
def test_vector_entry_points_refuse_bad_tensors(ctx, k):
    bad, exc = _bad_vectors()[k]
    calls = [
        lambda: ctx.residual(0, bad, bad),
        lambda: ctx.relax([0], [bad], [bad]),
        lambda: ctx.gmres([0], [bad], [bad]),
        lambda: ctx.rk_harmonic(0, bad, bad, 1),
        lambda: _net(ctx).apply(0, bad),
        lambda: _net(ctx).loss_grad([0], [bad], [bad]),
        lambda: _net(ctx).add_pairs([0], [bad], [bad]),
    ]
    for call in calls:
        with pytest.raises(exc):
            call()


@pytest.mark.parametrize("k", range(4))
def test_state_entry_points_refuse_bad_tensors(ctx, k):
    bad, exc = _bad_states()[k]
    for call in (lambda: ctx.assemble_jacobian(bad),
                 lambda: ctx.rusanov_residual(bad),
                 lambda: ctx.rk_mean(0, bad, 1)):
        with pytest.raises(exc):
            call()


def test_block_entry_point_refuses_bad_tensors(ctx):
    with pytest.raises(TypeError):
        ctx.set_blocks(torch.zeros((N, 6, 6), dtype=torch.float32), torch.zeros((E, 2, 6, 6), dtype=torch.float32))
    with pytest.raises(ValueError):
        ctx.set_blocks(torch.zeros((N, 6, 5), dtype=torch.float64), torch.zeros((E, 2, 6, 6), dtype=torch.float64))
    with pytest.raises(TypeError):   # right dtype and shape, host memory
        ctx.set_blocks(torch.zeros((N, 6, 6), dtype=torch.float64), torch.zeros((E, 2, 6, 6), dtype=torch.float64))


def test_count_mismatch_refused(ctx):
    with pytest.raises(ValueError):
        ctx.relax([0, 1], [], [])
    with pytest.raises(ValueError):
        _net(ctx).loss_grad([0, 1], [], [])


@pytest.mark.gpu
def test_device_index_checked(ctx):
    """A tensor on another device than the context's is refused before any call."""
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx.device = 1
    x = torch.zeros(VEC, dtype=torch.complex128, device="cuda:0")
    with pytest.raises(ValueError):
        ctx.residual(0, x, x)
    with pytest.raises(ValueError):
        ctx.relax([0], [x], [x])


def test_one_hip_runtime_whatever_the_import_order():
    """Importing the binding before torch must still leave one HIP runtime in the process
    (torch's): two runtimes side by side leave the library without a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import paper_2404_01407_amd.fnlh\nimport torch\n"
            "print('\\n'.join(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l})))")
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    libs = out.stdout.split()
    assert len(libs) == 1, libs
    assert os.path.realpath(libs[0]).startswith(os.path.realpath(os.path.dirname(torch.__file__))), libs
