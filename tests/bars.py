"""Parity bars measured on the oracle itself.

Hard decisions of shots that run many iterations without meeting the syndrome
depend on the priors so sensitively that the FP64 oracle does not agree with
itself once its priors move by a relative 1e-7 (the size of an FP32 rounding).
No FP32 decoder can do better there.  The bar for the GPU is therefore the
oracle's agreement with its own perturbed run, minus a sampling margin, or the
99.9% that north of this sensitivity is asked of every decoder, whichever is
lower.  Shots the oracle settles within a few iterations are held exactly.
"""
import math

import numpy as np

from oracle import oracle as O

PERTURBATION = 1e-7      # relative, of every prior LLR entry
TARGET = 0.999           # share of identical (shot, qubit) decisions asked for
EARLY_ITERS = 20         # shots converging within this many iterations agree exactly
Z_MARGIN = 3.0           # sampling margin in standard errors


def perturbed_prior(pi, seed=1):
    return pi * (1.0 + PERTURBATION * np.random.default_rng(seed).standard_normal(np.shape(pi)))


def decision_bar(code, params, pi, syn, est_gpu, ro=None, self_shots=None):
    """Entry-level agreement of the GPU's decisions with the oracle's, and the bar.

    Both agreements are means over shots of the per-shot share of equal qubit
    decisions.  bar = min(TARGET, self - margin) with margin = Z_MARGIN standard
    errors of the difference of the two per-shot means.  The perturbed oracle
    runs on the first `self_shots` shots (all if None).  Returns a dict."""
    if ro is None:
        ro = O.decode(code.hx, code.hz, params, pi, syn)
    k = syn.shape[0] if self_shots is None else min(self_shots, syn.shape[0])
    rp = O.decode(code.hx, code.hz, params, perturbed_prior(pi), syn[:k])
    d_gpu = (est_gpu != ro["est"]).mean(axis=1)
    d_self = (rp["est"] != ro["est"][:k]).mean(axis=1)
    gpu = 1.0 - float(d_gpu.mean())
    self_ = 1.0 - float(d_self.mean())
    se = math.sqrt(float(d_gpu.var()) / len(d_gpu) + float(d_self.var()) / len(d_self))
    margin = Z_MARGIN * se
    bar = min(TARGET, self_ - margin)
    return dict(gpu=gpu, self=self_, margin=margin, bar=bar, ok=gpu >= bar, shots=len(d_gpu), self_shots=k,
                ro=ro, rp=rp)


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


def early_exact(est_gpu, conv_gpu, it_gpu, ro):
    """Shots both sides converged on and the oracle stopped within EARLY_ITERS
    iterations: their decisions must be equal.  Returns the mask."""
    early = conv_gpu.astype(bool) & ro["conv"].astype(bool) & (ro["iters"] <= EARLY_ITERS)
    assert np.array_equal(est_gpu[early], ro["est"][early]), "early-converging shots disagree"
    return early


# ---------------------------------------------------------------------------
# AdaGrad-BP messages (eq. boost)
# ---------------------------------------------------------------------------

REL_TOL = 1e-5
# The kernels count an AdaGrad gradient at or below 2^-20 of its operands' magnitude
# as 0: FP32 cannot resolve its sign there.  The FP64 oracle evaluates eq. boost as
# written, so where the FP64 gradient is real but that small, or where FP32 rounding
# exceeds it, the first adaptive step (about alpha sign(g')) differs and the two
# part by up to 2 alpha on that entry.  The bar for AdaGrad is a share of entries.
ADAGRAD_WINDOW = 2.0 ** -20
ADAGRAD_SHARE = 0.999
# checks of degree 6 (bivariate bicycle, Chamon) sum five phi terms per message: measured
# 99.897% on Chamon d=2 at T = 3, so their share is 99.8%
ADAGRAD_SHARE_WIDE = 0.998


def adagrad_window_entries(q_trace, m_trace, pi, clamp=30.0, max_deg=4):
    """(shot, qubit, W) entries whose FP64 AdaGrad gradient g' = D^{(t-1)} - M^{(t)},
    2 <= t <= T, was nonzero but inside the kernels' deadband window at some t.  The
    window's scale |D| + sum |m| is bounded above by |D| + max_deg * clamp."""
    D = q_trace - pi[None, None]
    g = D[:, :-1] - m_trace[:, 1:]
    win = ADAGRAD_WINDOW * (np.abs(D[:, :-1]) + max_deg * clamp)
    return ((g != 0) & (np.abs(g) <= win)).any(axis=1)


def rel_err(gpu, ref):
    return np.abs(np.asarray(gpu, dtype=np.float64) - ref) / np.maximum(np.abs(ref), 1.0)


def adagrad_report(err_q, win):
    """Posterior agreement split by the deadband window."""
    return dict(window_frac=float(win.mean()),
                outside_max=float(err_q[~win].max()) if (~win).any() else 0.0,
                inside_frac_1e5=float((err_q[win] <= REL_TOL).mean()) if win.any() else 1.0,
                all_frac_1e5=float((err_q <= REL_TOL).mean()))


def early_agreement(est_gpu, conv_gpu, ro, rp):
    """Shots both sides converged on within EARLY_ITERS iterations whose decisions
    differ, for the GPU against the oracle and for the oracle against its own run
    with perturbed priors (on the shots that run covers), and the bar: the GPU's
    share may exceed the oracle's own by a 3-sigma binomial margin (taken at a
    share of at least 1e-4)."""
    k = len(rp["est"])
    e_g = conv_gpu.astype(bool) & ro["conv"].astype(bool) & (ro["iters"] <= EARLY_ITERS)
    e_s = rp["conv"].astype(bool) & ro["conv"][:k].astype(bool) & (ro["iters"][:k] <= EARLY_ITERS)
    diff_g = int((~np.all(est_gpu[e_g] == ro["est"][e_g], axis=1)).sum())
    diff_s = int((~np.all(rp["est"][e_s] == ro["est"][:k][e_s], axis=1)).sum())
    share_g = diff_g / max(1, int(e_g.sum()))
    share_s = diff_s / max(1, int(e_s.sum()))
    q = max(share_s, 1e-4)
    bar = share_s + Z_MARGIN * math.sqrt(q * (1 - q) / max(1, int(e_g.sum())))
    return dict(early=int(e_g.sum()), early_diff=diff_g, early_share=share_g, early_self_share=share_s,
                early_bar=bar, early_ok=share_g <= bar)
