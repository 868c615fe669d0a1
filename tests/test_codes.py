"""Pins of the workload generators (section II-A): code parameters, commutation,
degrees, logical bases and small distances by brute force."""
import itertools
import json
import os

import numpy as np
import pytest

import qecgen
from qecgen import gf2_rank, symplectic_product

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("L", [3, 5, 7, 9, 11, 13])
def test_planar_parameters(L):
    c = qecgen.planar(L)
    # [[2L^2 - 2L + 1, 1, L]] (section II-A)
    assert c.n == 2 * L * L - 2 * L + 1
    assert c.k == 1
    assert c.m == 2 * L * (L - 1)
    assert c.nnz == 4 * (L - 1) * (2 * L - 1)


@pytest.mark.parametrize("L", [3, 4, 6, 8, 10, 14])
def test_toric_parameters(L):
    c = qecgen.toric(L)
    # [[2L^2, 2, L]] (section II-A); every stabilizer has weight four (section IV-B2)
    assert c.n == 2 * L * L and c.m == 2 * L * L
    assert c.k == 2
    assert np.all((c.labels() > 0).sum(axis=1) == 4)
    assert np.all((c.labels() > 0).sum(axis=0) == 4)


@pytest.mark.parametrize("L,k", [(3, 1), (4, 2), (5, 1), (6, 2), (9, 1), (13, 1)])
def test_xzzx_parameters(L, k):
    c = qecgen.xzzx(L)
    assert c.n == L * L
    assert c.k == k
    lab = c.labels()
    for row in lab:
        nz = row[row > 0]
        assert sorted(nz.tolist()) == [1, 1, 2, 2]  # X Z Z X


@pytest.mark.parametrize("make", [lambda: qecgen.planar(3), lambda: qecgen.planar(5),
                                  lambda: qecgen.toric(4), lambda: qecgen.xzzx(5),
                                  lambda: qecgen.xzzx(4), lambda: qecgen.trapping_ring()])
def test_stabilizers_commute_and_logicals_are_symplectic(make):
    c = make()
    assert not symplectic_product(c.hx, c.hz, c.hx, c.hz).any()
    k = c.k
    assert c.lx.shape == (2 * k, c.n)
    assert not symplectic_product(c.hx, c.hz, c.lx, c.lz).any()
    gram = symplectic_product(c.lx, c.lz, c.lx, c.lz)
    want = np.block([[np.zeros((k, k)), np.eye(k)], [np.eye(k), np.zeros((k, k))]])
    assert np.array_equal(gram, want)
    stacked = np.vstack([np.hstack([c.hx, c.hz]), np.hstack([c.lx, c.lz])])
    assert gf2_rank(stacked) == c.rank + 2 * k  # logicals are outside the stabilizer group


def _distance(c, wmax):
    """Minimum weight of a Pauli that commutes with S and is not in S (brute force)."""
    n = c.n
    sx, sz = c.hx.astype(np.int64), c.hz.astype(np.int64)
    lx, lz = c.lx.astype(np.int64), c.lz.astype(np.int64)
    for w in range(1, wmax + 1):
        for supp in itertools.combinations(range(n), w):
            for ps in itertools.product((1, 2, 3), repeat=w):
                ex = np.zeros(n, np.int64)
                ez = np.zeros(n, np.int64)
                for q, p in zip(supp, ps):
                    ex[q] = p & 1
                    ez[q] = p >> 1
                if ((sx @ ez + sz @ ex) & 1).any():
                    continue
                if ((lx @ ez + lz @ ex) & 1).any():
                    return w
    return None


@pytest.mark.parametrize("make,d", [(lambda: qecgen.planar(3), 3), (lambda: qecgen.toric(3), 3),
                                    (lambda: qecgen.xzzx(3), 3)])
def test_small_distances(make, d):
    assert _distance(make(), d) == d


def test_trapping_set_syndrome_matches_paper():
    # Section IV-A: X errors on qubits 1 and 2 of the (4,0) trapping set give [1,0,1,0].
    g = _golden()["trapping_set"]
    c = qecgen.trapping_ring()
    e = np.zeros(4, np.uint8)
    for q in g["x_error_qubits_1based"]:
        e[q - 1] = 1
    s = symplectic_product(c.hx, c.hz, e & 1, e >> 1)[:, 0]
    assert s.tolist() == g["syndrome"]


def test_thresholds_and_probs():
    t = qecgen.thresholds(0.1 / 3, 0.1 / 3, 0.1 / 3)
    assert t.dtype == np.uint32 and abs(int(t[0]) - round(2 ** 32 * 0.1 / 3)) == 0
    with pytest.raises(ValueError):
        qecgen.thresholds(0.5, 0.3, 0.3)
    b = qecgen.biased_probs(3, 0.06)
    assert np.allclose(b.sum(axis=1), 0.06) and np.allclose(b[:, 2], 0.04)
