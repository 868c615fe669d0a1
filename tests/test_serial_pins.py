"""Pins of the oracle's serial schedule (Algorithm 1: qubit by qubit in index order,
each qubit's incoming check messages recomputed from the current messages of the
check's other qubits, then its posterior and outgoing messages).

* on cycle-free graphs the serial schedule also reaches the exact marginals
  (brute force over 4^n errors);
* on graphs with cycles it equals an independent probability-domain quaternary BP
  run in the same serial order (4-vector messages, explicit sums over neighbour
  configurations), for BP, EWAInit and Momentum (gamma = 0), with Y labels;
* the schedule matters: after one iteration serial and flooding differ.
"""
import itertools
import math

import numpy as np
import pytest

import qecgen
from oracle import oracle as O
from tests.test_oracle_pins import COMM, brute_force_llr, clifford_relabel, random_forest, syndrome_np


@pytest.mark.parametrize("seed", range(8))
def test_serial_tree_exact_marginals(seed):
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(4, 8))
    hx, hz = random_forest(n, int(rng.integers(2, n)), rng)
    m = hx.shape[0]
    probs = rng.dirichlet([8, 1, 1, 1], size=n)[:, 1:]
    allE = np.array(list(itertools.product(range(4), repeat=n)), dtype=np.uint8)
    pfull = np.column_stack([1 - probs.sum(1), probs[:, 0], probs[:, 2], probs[:, 1]])
    P = np.prod(pfull[np.arange(n), allE], axis=1)
    e0 = allE[rng.choice(len(allE), p=P / P.sum())]
    s = syndrome_np(hx, hz, e0)[0]
    Qb, _, _ = brute_force_llr(hx, hz, probs, s)
    r = O.decode(hx, hz, O.Params(variant="bp", max_iter=2 * (n + m), stop_on_syndrome=False, clamp=math.inf,
                                  serial=True), O.prior_llr(probs), s[None], want_q=True)
    assert np.allclose(r["q"][0], Qb, rtol=1e-10, atol=1e-10)


def prob_bp4_serial(hx, hz, probs, s, T, variant="bp", alpha=1.0):
    """Quaternary sum-product in the serial order of Algorithm 1, probability domain."""
    m, n = hx.shape
    lab = (hx | (hz << 1)).astype(int)
    edges = [(c, v) for c in range(m) for v in range(n) if lab[c, v]]
    p0 = np.column_stack([1 - probs.sum(1), probs[:, 0], probs[:, 2], probs[:, 1]])
    q = {e: p0[e[1]].copy() for e in edges}
    post_prev = p0.copy()
    out = []
    for t in range(1, T + 1):
        prior = p0.copy()
        if variant == "ewainit" and t > 1:
            prior = p0 ** alpha * post_prev ** (1 - alpha)
            prior /= prior.sum(1, keepdims=True)
        base = p0 if variant in ("bp", "momentum") else prior
        post = np.zeros_like(p0)
        for v in range(n):
            checks = [c for c in range(m) if lab[c, v]]
            r = {}
            for c in checks:
                others = [u for u in range(n) if lab[c, u] and u != v]
                rv = np.zeros(4)
                for Pv in range(4):
                    tot = 0.0
                    for conf in itertools.product(range(4), repeat=len(others)):
                        par = COMM[lab[c, v], Pv]
                        w = 1.0
                        for u, Pu in zip(others, conf):
                            par ^= COMM[lab[c, u], Pu]
                            w *= q[(c, u)][Pu]
                        if par == s[c]:
                            tot += w
                    rv[Pv] = tot
                r[c] = rv / rv.sum()
            pv = base[v].copy()
            for c in checks:
                pv = pv * r[c]
            pv /= pv.sum()
            if variant == "momentum":
                pv = pv ** alpha * post_prev[v] ** (1 - alpha)
                pv /= pv.sum()
            post[v] = pv
            for c in checks:
                if variant == "momentum":
                    qq = pv / r[c]
                else:
                    qq = base[v].copy()
                    for c2 in checks:
                        if c2 != c:
                            qq = qq * r[c2]
                q[(c, v)] = qq / qq.sum()
        post_prev = post
        out.append(np.log(post[:, [0]]) - np.log(post[:, [1, 3, 2]]))
    return np.array(out)


@pytest.mark.parametrize("make", [lambda: qecgen.planar(3), lambda: qecgen.toric(3), lambda: qecgen.xzzx(3)])
@pytest.mark.parametrize("variant,alpha", [("bp", 1.0), ("ewainit", 0.6), ("momentum", 0.7)])
def test_serial_probability_domain(make, variant, alpha):
    code = make()
    rng = np.random.default_rng(6)
    hx, hz, _ = clifford_relabel(code, rng)
    probs = rng.uniform(0.005, 0.04, size=(code.n, 3))
    e = np.zeros(code.n, np.uint8)
    e[rng.choice(code.n, 2, replace=False)] = rng.integers(1, 4, size=2)
    s = syndrome_np(hx, hz, e)[0]
    T = 5
    want = prob_bp4_serial(hx, hz, probs, s, T, variant, alpha)
    r = O.decode(hx, hz, O.Params(variant=variant, max_iter=T, stop_on_syndrome=False, clamp=math.inf,
                                  alpha=alpha, serial=True), O.prior_llr(probs), s[None], want_trace=True)
    assert np.allclose(r["q_trace"][0], want, rtol=1e-9, atol=1e-9)
    flood = O.decode(hx, hz, O.Params(variant=variant, max_iter=T, stop_on_syndrome=False, clamp=math.inf,
                                      alpha=alpha), O.prior_llr(probs), s[None], want_trace=True)
    assert not np.allclose(flood["q_trace"][0][0], r["q_trace"][0][0], rtol=1e-6, atol=1e-6)
