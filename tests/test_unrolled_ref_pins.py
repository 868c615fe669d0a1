"""Pins of the FP64 reference for the unrolled EWAInit loss and its gradient (CPU).

The reference (oracle/unrolled_ref.py, torch float64 autograd) is pinned to the
C oracle, which is independent code with its own pins: its posterior Q^{(T)}
must equal the C oracle's to 1e-12 (per-iteration discounts, Y labels,
non-uniform priors, with and without clamping), and its gradient must equal
central finite differences of the C oracle's loss to 1e-7 relative.  A planted
mistake in the reference (a dropped term, a wrong sign or index) moves one of
these far beyond the bar.
"""
import numpy as np
import pytest

import qecgen
from oracle import oracle as O
from oracle import unrolled_ref as U


def clifford_relabel(code, rng):
    lab = code.labels()
    new = np.zeros_like(lab)
    for v in range(code.n):
        p = rng.permutation([1, 2, 3])
        mp = np.array([0, p[0], p[1], p[2]], np.uint8)
        new[:, v] = mp[lab[:, v]]
    return (new & 1).astype(np.uint8), (new >> 1).astype(np.uint8)


def _case(name, seed):
    rng = np.random.default_rng(seed)
    if name == "planar3":
        c = qecgen.planar(3)
        hx, hz = c.hx, c.hz
    elif name == "toric3":
        c = qecgen.toric(3)
        hx, hz = c.hx, c.hz
    else:
        c = qecgen.xzzx(3)
        hx, hz = clifford_relabel(c, rng)
    n = c.n
    probs = rng.uniform(0.02, 0.05, size=(n, 3))
    prior = O.prior_llr(probs)
    err, syn = O.sample(hx, hz, 48, qecgen.thresholds(0.035, 0.03, 0.04), seed=seed)
    return hx, hz, prior, err, syn, rng


def _oracle_q(hx, hz, alpha, prior, syn, T, clamp):
    p = O.Params(variant="ewainit", max_iter=T, stop_on_syndrome=False, alpha_t=alpha, clamp=clamp)
    return O.decode(hx, hz, p, prior, syn, want_q=True)["q"]


@pytest.mark.parametrize("name", ["planar3", "toric3", "xzzx3-clifford"])
@pytest.mark.parametrize("clamp", [30.0, float("inf")])
def test_reference_forward_equals_c_oracle(name, clamp):
    hx, hz, prior, err, syn, rng = _case(name, 5)
    T = 7
    alpha = rng.uniform(0.2, 0.95, T)
    L, _, _, Q = U.loss_and_grad(hx, hz, alpha, prior, syn, err, T, clamp)
    q = _oracle_q(hx, hz, alpha, prior, syn, T, clamp)
    assert np.max(np.abs(Q - q) / np.maximum(np.abs(q), 1.0)) <= 1e-12
    assert abs(L - U.soft_loss(q, err)) <= 1e-12 * max(1.0, abs(L))


@pytest.mark.parametrize("name", ["planar3", "xzzx3-clifford"])
def test_reference_gradient_equals_finite_differences_of_c_oracle(name):
    # clamp off, so the loss is smooth at the evaluation point (no active clamp)
    hx, hz, prior, err, syn, rng = _case(name, 9)
    T = 6
    alpha = rng.uniform(0.3, 0.9, T)
    inf = float("inf")
    _, ga, gp, _ = U.loss_and_grad(hx, hz, alpha, prior, syn, err, T, inf)

    def loss(a, p):
        return U.soft_loss(_oracle_q(hx, hz, a, p, syn, T, inf), err)

    fa = np.zeros(T)
    for t in range(1, T):          # alpha_1 is unused: its gradient is 0
        h = 1e-6 * max(1.0, abs(alpha[t]))
        ap, am = alpha.copy(), alpha.copy()
        ap[t] += h
        am[t] -= h
        fa[t] = (loss(ap, prior) - loss(am, prior)) / (2 * h)
    fp = np.zeros_like(prior)
    for i in range(prior.shape[0]):
        for w in range(3):
            h = 1e-6 * max(1.0, abs(prior[i, w]))
            pp, pm = prior.copy(), prior.copy()
            pp[i, w] += h
            pm[i, w] -= h
            fp[i, w] = (loss(alpha, pp) - loss(alpha, pm)) / (2 * h)
    assert ga[0] == 0.0
    # central differences carry ~1e-16 |L| / h = 1e-11 of rounding noise, so each
    # element is held to 1e-7 of itself or of 1% of the largest element
    for g, f in ((ga, fa), (gp, fp)):
        floor = 1e-2 * np.max(np.abs(g))
        assert np.max(np.abs(g - f) / np.maximum(np.abs(g), floor)) <= 1e-7


def test_reference_alpha_one_is_traditional_bp():
    # alpha_t = 1: Pi^{(t)} = Pi^{(0)} at every iteration, the C oracle's traditional BP
    hx, hz, prior, err, syn, rng = _case("planar3", 2)
    T = 5
    _, _, _, Q = U.loss_and_grad(hx, hz, np.ones(T), prior, syn, err, T)
    q = O.decode(hx, hz, O.Params(variant="bp", max_iter=T, stop_on_syndrome=False), prior, syn,
                 want_q=True)["q"]
    assert np.max(np.abs(Q - q) / np.maximum(np.abs(q), 1.0)) <= 1e-12
