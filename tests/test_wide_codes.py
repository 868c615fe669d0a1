"""Codes with checks and qubits of degree 6 (section IV-C: bivariate bicycle codes and
3D Chamon codes), their constructions and the FP64 oracle on such graphs.

* the bivariate bicycle instances reproduce the published parameters k (12, 8, 8, 12,
  12 for n = 72, 90, 108, 144, 288); the Chamon code on the (2d)^3 lattice has
  k = 4 gcd(d, d, d) = 4d; every check and qubit has weight 6; all stabilizers commute;
* the oracle on cycle-free graphs with checks of degree up to 6 reaches the exact
  marginals (brute force over 4^n errors);
* the oracle on the Chamon d=2 code (degree 6, Y labels) equals the independent
  probability-domain quaternary BP.
"""
import itertools
import math

import numpy as np
import pytest

import qecgen
from oracle import oracle as O
from tests.test_oracle_pins import brute_force_llr, prob_bp4, syndrome_np


@pytest.mark.parametrize("n,k", [(72, 12), (90, 8), (108, 8), (144, 12), (288, 12)])
def test_bivariate_bicycle_parameters(n, k):
    c = qecgen.bb(n)
    lab = c.labels()
    assert c.n == n and c.k == k
    assert set((lab != 0).sum(1)) == {6} and set((lab != 0).sum(0)) == {6}
    assert not qecgen.symplectic_product(c.hx, c.hz, c.hx, c.hz).any()
    # logical basis: symplectic pairs, commuting with every stabilizer
    g = qecgen.symplectic_product(c.lx, c.lz, c.lx, c.lz)
    kk = c.lx.shape[0] // 2
    assert kk == k
    want = np.zeros((2 * k, 2 * k), np.uint8)
    want[:k, k:] = np.eye(k, dtype=np.uint8)
    want[k:, :k] = np.eye(k, dtype=np.uint8)
    assert np.array_equal(g, want)
    assert not qecgen.symplectic_product(c.lx, c.lz, c.hx, c.hz).any()


@pytest.mark.parametrize("d", [2, 3, 4])
def test_chamon_parameters(d):
    c = qecgen.chamon(d)
    lab = c.labels()
    assert c.n == 4 * d ** 3 and c.m == 4 * d ** 3
    assert c.k == 4 * d
    assert set((lab != 0).sum(1)) == {6} and set((lab != 0).sum(0)) == {6}
    assert (lab == 3).any() and (lab == 1).any() and (lab == 2).any()   # X, Y and Z entries
    assert not qecgen.symplectic_product(c.hx, c.hz, c.hx, c.hz).any()


def wide_forest(n, rng):
    """A random cycle-free Tanner graph with checks of degree 2 ... 6 and GF(4) labels."""
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            a = parent[a]
        return a

    rows = []
    for it in range(1000):
        d = int(rng.integers(5, 7)) if it == 0 else int(rng.integers(2, 7))   # one wide check first
        if d > n:
            continue
        vs = rng.choice(n, size=d, replace=False)
        roots = [find(int(v)) for v in vs]
        if len(set(roots)) < d:
            continue
        for r in roots[1:]:
            parent[r] = roots[0]
        rows.append((vs, rng.integers(1, 4, size=d)))
        if len(set(find(v) for v in range(n))) == 1:
            break
    hx = np.zeros((len(rows), n), np.uint8)
    hz = np.zeros_like(hx)
    for i, (vs, ls) in enumerate(rows):
        for v, l in zip(vs, ls):
            hx[i, v] = l & 1
            hz[i, v] = l >> 1
    return hx, hz


@pytest.mark.parametrize("seed", range(6))
def test_wide_tree_exact_marginals(seed):
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(6, 9))
    hx, hz = wide_forest(n, rng)
    assert ((hx | hz) != 0).sum(1).max() >= 5
    m = hx.shape[0]
    probs = rng.dirichlet([8, 1, 1, 1], size=n)[:, 1:]
    allE = np.array(list(itertools.product(range(4), repeat=n)), dtype=np.uint8)
    pfull = np.column_stack([1 - probs.sum(1), probs[:, 0], probs[:, 2], probs[:, 1]])
    P = np.prod(pfull[np.arange(n), allE], axis=1)
    e0 = allE[rng.choice(len(allE), p=P / P.sum())]
    s = syndrome_np(hx, hz, e0)[0]
    Qb, _, _ = brute_force_llr(hx, hz, probs, s)
    r = O.decode(hx, hz, O.Params(variant="bp", max_iter=2 * (n + m), stop_on_syndrome=False, clamp=math.inf),
                 O.prior_llr(probs), s[None], want_q=True)
    assert np.allclose(r["q"][0], Qb, rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("variant,alpha", [("bp", 1.0), ("ewainit", 0.6)])
def test_chamon_probability_domain_bp4(variant, alpha):
    c = qecgen.chamon(2)
    rng = np.random.default_rng(9)
    probs = rng.uniform(0.005, 0.04, size=(c.n, 3))
    e = np.zeros(c.n, np.uint8)
    e[rng.choice(c.n, 2, replace=False)] = rng.integers(1, 4, size=2)
    s = syndrome_np(c.hx, c.hz, e)[0]
    T = 3
    want = prob_bp4(c.hx, c.hz, probs, s, T, variant, alpha)
    r = O.decode(c.hx, c.hz, O.Params(variant=variant, max_iter=T, stop_on_syndrome=False, clamp=math.inf,
                                      alpha=alpha), O.prior_llr(probs), s[None], want_trace=True)
    assert np.allclose(r["q_trace"][0], want, rtol=1e-9, atol=1e-9)
