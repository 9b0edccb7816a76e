"""Shared helpers for the GPU parity tests: build cases from the seeded generator, move
data to the device, run the oracle with the GPU's colouring."""
import numpy as np

from oracle import assemble, precision, solve
from paper_2404_01407_amd import synth


def case(shape=(16, 8, 4), n_blades=36, seed=1, sigma=50.0, jitter=0.1):
    m = synth.passage_block(*shape, n_blades, seed=seed, jitter=jitter)
    Q = synth.flow_state(m, seed)
    K = assemble.assemble(m, Q, sigma=sigma)
    return m, Q, K


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def blocks_user_layout(K):
    """Oracle BlockMatrix -> (diag [N,6,6], offd [E,2,6,6]) in the set_blocks layout."""
    E = K.offd.shape[0] // 2
    offd = np.stack([K.offd[0::2], K.offd[1::2]], axis=1)
    return np.ascontiguousarray(K.diag), np.ascontiguousarray(offd.reshape(E, 2, 6, 6))


def rounded(K, storage):
    Kr = K.copy()
    Kr.diag = precision.round_storage(K.diag, storage)
    Kr.offd = precision.round_storage(K.offd, storage)
    return Kr


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rowerr(a, b):
    """Worst single entry: max over rows i and the six components k of
    |a_ik - b_ik| / rms_i |b_ik|.  Each component is measured against its own scale, so a
    small component (the turbulence variable) or a handful of rows (boundary cells)
    cannot hide behind the norm of the whole field."""
    a = np.asarray(a).reshape(-1, 6)
    b = np.asarray(b).reshape(-1, 6)
    rms = np.sqrt(np.mean(np.abs(b) ** 2, axis=0))
    return float(np.max(np.abs(a - b) / np.maximum(rms, 1e-300)))


def itererr(a, b):
    """Iterate parity: the larger of the field's relative error and the per-row,
    per-component error of rowerr."""
    return max(relerr(a, b), rowerr(a, b))
