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


def decision_margin(code, params, pi0, syn_row, t):
    """Smallest distance, over the qubits, of the oracle's FP64 posterior LLRs at
    iteration t from a change of the hard decision (section II-B1: identity when
    every LLR is positive, else the smallest one).  An FP32 decoder can only take
    a different decision where this is at rounding level."""
    r = O.decode(code.hx, code.hz, params, pi0, syn_row.reshape(1, -1), want_trace=True)
    q = np.sort(r["q_trace"][0, t - 1], axis=1)
    margin = np.where(q[:, 0] > 0, q[:, 0], np.minimum(-q[:, 0], q[:, 1] - q[:, 0]))
    scale = np.maximum(1.0, np.abs(q).max(axis=1))
    return float((margin / scale).min())


def same_stops(code, params, pi0, syn, it_a, it_b, rel=1e-3):
    """Shots whose stopping iterations differ are accepted only where the FP64
    decision at the earlier of the two iterations is within `rel` of a tie.
    Returns the indices of the differing shots and their margins."""
    bad = np.nonzero(it_a != it_b)[0]
    margins = [decision_margin(code, params, pi0, syn[i], int(min(it_a[i], it_b[i]))) for i in bad]
    assert all(m <= rel for m in margins), (bad, margins)
    return bad, margins
