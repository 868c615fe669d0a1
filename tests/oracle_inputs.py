"""The oracle's own errors and syndromes for shots the GPU also sampled.

A GPU test that checks decoded shots against the oracle hands the oracle inputs
drawn by the oracle's sampler (the same Philox streams, keyed by seed and shot
index), never rows read back from the GPU, and asserts that the GPU's rows are
bit-identical to them.
"""
import numpy as np

from oracle import oracle as O


def rows(code, thr, seed, idx=None, shots=None):
    """Errors and syndromes of the shots `idx` (or of shots 0..shots-1)."""
    if idx is None:
        return O.sample(code.hx, code.hz, shots, thr, seed=seed)
    es, ss = zip(*(O.sample(code.hx, code.hz, 1, thr, seed=seed, shot0=int(i)) for i in idx))
    return np.concatenate(es), np.concatenate(ss)


def matched(code, thr, seed, err_gpu, syn_gpu, idx=None):
    """The oracle's rows for the GPU batch (all shots, or those in `idx`),
    checked bit for bit against the GPU sampler's rows."""
    if idx is None:
        e, s = rows(code, thr, seed, shots=syn_gpu.shape[0])
        ge, gs = err_gpu.cpu().numpy(), syn_gpu.cpu().numpy()
    else:
        e, s = rows(code, thr, seed, idx=idx)
        import torch
        sel = torch.as_tensor(np.asarray(idx), device=syn_gpu.device)
        ge, gs = err_gpu[sel].cpu().numpy(), syn_gpu[sel].cpu().numpy()
    assert np.array_equal(gs, s), "GPU syndromes differ from the oracle's sampler"
    assert np.array_equal(ge, e), "GPU errors differ from the oracle's sampler"
    return e, s
