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
