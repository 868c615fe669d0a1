"""Pins of the FP64 reference for the unrolled EWAInit and Momentum loss and its gradient (CPU).

The reference (oracle/unrolled_ref.py, torch float64 autograd) is pinned to the
C oracle, which is independent code with its own pins: its posterior Q^{(T)}
must equal the C oracle's to 1e-12 (per-iteration discounts, Momentum steps and
decays, Y labels, non-uniform priors, with and without clamping), and its
gradient must equal central finite differences of the C oracle's loss to 1e-7
relative.  Special cases reduce both variants to traditional BP.  A planted
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


# ---------------------------------------------------------------------------
# Momentum-BP with a step alpha_t and a decay gamma_t per iteration (section III-A1,
# eqs. mombp1-3): params [T, 2]
# ---------------------------------------------------------------------------

def _oracle_q_momentum(hx, hz, params, prior, syn, T, clamp):
    p = O.Params(variant="momentum", max_iter=T, stop_on_syndrome=False, alpha_t=params[:, 0],
                 gamma_t=params[:, 1], clamp=clamp)
    return O.decode(hx, hz, p, prior, syn, want_q=True)["q"]


def _momentum_params(rng, T):
    return np.stack([rng.uniform(0.3, 1.0, T), rng.uniform(0.0, 0.8, T)], axis=1)


@pytest.mark.parametrize("name", ["planar3", "toric3", "xzzx3-clifford"])
@pytest.mark.parametrize("clamp", [30.0, float("inf")])
def test_reference_momentum_forward_equals_c_oracle(name, clamp):
    hx, hz, prior, err, syn, rng = _case(name, 15)
    T = 7
    params = _momentum_params(rng, T)
    L, _, _, Q = U.loss_and_grad(hx, hz, params, prior, syn, err, T, clamp, variant="momentum")
    q = _oracle_q_momentum(hx, hz, params, prior, syn, T, clamp)
    assert np.max(np.abs(Q - q) / np.maximum(np.abs(q), 1.0)) <= 1e-12
    assert abs(L - U.soft_loss(q, err)) <= 1e-12 * max(1.0, abs(L))
    # the per-iteration parameters are used: constant ones give another posterior
    q_const = O.decode(hx, hz, O.Params(variant="momentum", max_iter=T, stop_on_syndrome=False,
                                        alpha=float(params[0, 0]), gamma=float(params[0, 1]), clamp=clamp),
                       prior, syn, want_q=True)["q"]
    assert np.max(np.abs(q_const - q)) > 1e-6


@pytest.mark.parametrize("name", ["planar3", "xzzx3-clifford"])
def test_reference_momentum_gradient_equals_finite_differences_of_c_oracle(name):
    hx, hz, prior, err, syn, rng = _case(name, 19)
    T = 6
    params = _momentum_params(rng, T)
    inf = float("inf")
    _, gpar, gp, _ = U.loss_and_grad(hx, hz, params, prior, syn, err, T, inf, variant="momentum")

    def loss(a, p):
        return U.soft_loss(_oracle_q_momentum(hx, hz, a, p, syn, T, inf), err)

    fpar = np.zeros_like(params)
    for t in range(T):
        for k in range(2):
            h = 1e-6 * max(1.0, abs(params[t, k]))
            ap, am = params.copy(), params.copy()
            ap[t, k] += h
            am[t, k] -= h
            fpar[t, k] = (loss(ap, prior) - loss(am, prior)) / (2 * h)
    fp = np.zeros_like(prior)
    for i in range(prior.shape[0]):
        for w in range(3):
            h = 1e-6 * max(1.0, abs(prior[i, w]))
            pp, pm = prior.copy(), prior.copy()
            pp[i, w] += h
            pm[i, w] -= h
            fp[i, w] = (loss(params, pp) - loss(params, pm)) / (2 * h)
    assert gpar.shape == (T, 2)
    for g, f in ((gpar, fpar), (gp, fp)):
        floor = 1e-2 * np.max(np.abs(g))
        assert np.max(np.abs(g - f) / np.maximum(np.abs(g), floor)) <= 1e-7


def test_reference_momentum_unit_step_no_decay_is_traditional_bp():
    # alpha_t = 1, gamma_t = 0: g^{(t)} = Q^{(t-1)} - Pi - M^{(t)}, so Q^{(t)} = Pi + M^{(t)}
    # (eq. p_update), and the messages lambda(Q) - m_{c->v} are BP's (eq. v_update)
    hx, hz, prior, err, syn, rng = _case("toric3", 3)
    T = 5
    params = np.stack([np.ones(T), np.zeros(T)], axis=1)
    _, _, _, Q = U.loss_and_grad(hx, hz, params, prior, syn, err, T, variant="momentum")
    q = O.decode(hx, hz, O.Params(variant="bp", max_iter=T, stop_on_syndrome=False), prior, syn,
                 want_q=True)["q"]
    assert np.max(np.abs(Q - q) / np.maximum(np.abs(q), 1.0)) <= 1e-12
