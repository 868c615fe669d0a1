"""Stabilizer codes used as decoder workloads, as symplectic check matrices.

Seeded-input module shared by the FP64 oracle tests and the GPU path: it builds
the check matrices and logical bases that describe a code, and holds none of
the decoding arithmetic.

Conventions
-----------
* A code on ``n`` qubits with ``m`` stabilizer rows is a pair ``(hx, hz)`` of
  ``uint8`` arrays of shape ``(m, n)``; row ``i`` is the Pauli
  ``prod_j X_j^{hx[i,j]} Z_j^{hz[i,j]}`` (Y where both bits are set).  This is the
  GF(4) check matrix of section II-B1: entry ``H_ij`` is the ``j``-th Pauli of
  stabilizer ``S_i``.
* The symplectic product of two Paulis ``(ax, az)`` and ``(bx, bz)`` is
  ``ax.bz + az.bx (mod 2)``; it is 1 exactly when they anticommute.

Families (section II-A):
* unrotated planar surface code ``[[2L^2-2L+1, 1, L]]`` (open boundaries),
* toric code ``[[2L^2, 2, L]]`` (periodic boundaries),
* XZZX surface code on an ``L x L`` torus, one ``X Z Z X`` face stabilizer per
  plaquette; even ``L`` gives ``K = 2`` as stated for this family, odd ``L``
  gives ``K = 1`` (the rank decides, see :func:`gf2_rank`).

Planar and toric codes are hypergraph products of the open and cyclic
repetition codes, the construction the paper names for the toric code in
section IV-B.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np


# ---------------------------------------------------------------------------
# GF(2) helpers
# ---------------------------------------------------------------------------

def _pack(a: np.ndarray) -> np.ndarray:
    """Pack 0/1 rows into uint64 words (bit j of the row in word j // 64)."""
    a = np.asarray(a, dtype=np.uint8) & 1
    rows, cols = a.shape
    words = (cols + 63) // 64
    pad = np.zeros((rows, words * 64), dtype=np.uint8)
    pad[:, :cols] = a
    bits = pad.reshape(rows, words, 64).astype(np.uint64)
    return (bits << np.arange(64, dtype=np.uint64)).sum(axis=2, dtype=np.uint64)


def _rref_packed(a: np.ndarray):
    """Reduced row echelon form over GF(2); returns (packed rows, pivot columns)."""
    a = np.asarray(a, dtype=np.uint8)
    rows, cols = a.shape
    p = _pack(a)
    pivots = []
    r = 0
    one = np.uint64(1)
    for c in range(cols):
        if r == rows:
            break
        w, b = divmod(c, 64)
        col = (p[r:, w] >> np.uint64(b)) & one
        nz = np.nonzero(col)[0]
        if nz.size == 0:
            continue
        piv = r + int(nz[0])
        if piv != r:
            p[[r, piv]] = p[[piv, r]]
        hit = np.nonzero((p[:, w] >> np.uint64(b)) & one)[0]
        hit = hit[hit != r]
        if hit.size:
            p[hit] ^= p[r]
        pivots.append(c)
        r += 1
    return p[:r], pivots


def _unpack_bit(p: np.ndarray, c: int) -> np.ndarray:
    w, b = divmod(c, 64)
    return ((p[:, w] >> np.uint64(b)) & np.uint64(1)).astype(np.uint8)


def gf2_rank(a: np.ndarray) -> int:
    """Rank over GF(2) of a 0/1 matrix."""
    return len(_rref_packed(a)[1])


def gf2_nullspace(a: np.ndarray) -> np.ndarray:
    """Basis (rows) of the right null space {v : a v = 0 mod 2}."""
    a = np.asarray(a, dtype=np.uint8)
    cols = a.shape[1]
    p, pivots = _rref_packed(a)
    pivset = set(pivots)
    free = [c for c in range(cols) if c not in pivset]
    basis = np.zeros((len(free), cols), dtype=np.uint8)
    piv_idx = np.array(pivots, dtype=np.int64)
    for k, f in enumerate(free):
        basis[k, f] = 1
        if len(pivots):
            basis[k, piv_idx] = _unpack_bit(p, f)
    return basis


def symplectic_product(ax, az, bx, bz) -> np.ndarray:
    """Pairwise symplectic products of row sets a (p x n) and b (q x n) -> (p x q)."""
    ax = np.atleast_2d(ax).astype(np.int64)
    az = np.atleast_2d(az).astype(np.int64)
    bx = np.atleast_2d(bx).astype(np.int64)
    bz = np.atleast_2d(bz).astype(np.int64)
    return ((ax @ bz.T + az @ bx.T) & 1).astype(np.uint8)


# ---------------------------------------------------------------------------
# Code container
# ---------------------------------------------------------------------------

@dataclass
class StabilizerCode:
    name: str
    hx: np.ndarray            # (m, n) uint8
    hz: np.ndarray            # (m, n) uint8
    lx: np.ndarray = field(default=None)  # (2k, n) uint8 logical basis, x part
    lz: np.ndarray = field(default=None)  # (2k, n) uint8 logical basis, z part
    coords: np.ndarray = field(default=None)  # (n, 2) int32 qubit positions on the layout, if the family has one

    @property
    def n(self) -> int:
        return int(self.hx.shape[1])

    @property
    def m(self) -> int:
        return int(self.hx.shape[0])

    @property
    def nnz(self) -> int:
        return int(np.count_nonzero(self.hx | self.hz))

    @property
    def rank(self) -> int:
        return gf2_rank(np.hstack([self.hx, self.hz]))

    @property
    def k(self) -> int:
        return self.n - self.rank

    def labels(self) -> np.ndarray:
        """GF(4) entries as Pauli codes, bit0 = x, bit1 = z (I=0, X=1, Z=2, Y=3)."""
        return (self.hx | (self.hz << 1)).astype(np.uint8)


def _finish(name: str, hx: np.ndarray, hz: np.ndarray, coords=None) -> StabilizerCode:
    hx = (np.asarray(hx) & 1).astype(np.uint8)
    hz = (np.asarray(hz) & 1).astype(np.uint8)
    code = StabilizerCode(name, hx, hz)
    code.lx, code.lz = logical_basis(hx, hz)
    if coords is not None:
        code.coords = np.asarray(coords, dtype=np.int32)
    return code


def _repetition_product_coords(n1: int, m1: int, n2: int, m2: int) -> np.ndarray:
    """Lattice positions of the qubits of a hypergraph product of two repetition codes
    (check r between bits r and r + 1): bit x bit qubit (i, j) at (2i, 2j), check x check
    qubit (a, b) at (2a + 1, 2b + 1), in the qubit order of hypergraph_product."""
    i, j = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
    a, b = np.meshgrid(np.arange(m1), np.arange(m2), indexing="ij")
    first = np.stack([2 * i.ravel(), 2 * j.ravel()], axis=1)
    second = np.stack([2 * a.ravel() + 1, 2 * b.ravel() + 1], axis=1)
    return np.vstack([first, second]).astype(np.int32)


# ---------------------------------------------------------------------------
# Families
# ---------------------------------------------------------------------------

def repetition_open(L: int) -> np.ndarray:
    """(L-1) x L parity checks of the open repetition code: rows e_r + e_{r+1}."""
    h = np.zeros((L - 1, L), dtype=np.uint8)
    for r in range(L - 1):
        h[r, r] = h[r, r + 1] = 1
    return h


def repetition_cyclic(L: int) -> np.ndarray:
    """L x L parity checks of the cyclic repetition code: rows e_r + e_{r+1 mod L}."""
    h = np.zeros((L, L), dtype=np.uint8)
    for r in range(L):
        h[r, r] = 1
        h[r, (r + 1) % L] = 1
    return h


def hypergraph_product(h1: np.ndarray, h2: np.ndarray):
    """CSS hypergraph product of classical checks h1 (m1 x n1) and h2 (m2 x n2).

    Qubits are the n1*n2 "bit x bit" block followed by the m1*m2 "check x check"
    block.  X checks: [h1 (x) I_n2 | I_m1 (x) h2^T]; Z checks: [I_n1 (x) h2 | h1^T (x) I_m2].
    Returns (hx, hz) stacked as [X rows; Z rows] over all qubits.
    """
    m1, n1 = h1.shape
    m2, n2 = h2.shape
    x_rows = np.hstack([np.kron(h1, np.eye(n2, dtype=np.uint8)),
                        np.kron(np.eye(m1, dtype=np.uint8), h2.T)]) & 1
    z_rows = np.hstack([np.kron(np.eye(n1, dtype=np.uint8), h2),
                        np.kron(h1.T, np.eye(m2, dtype=np.uint8))]) & 1
    n = n1 * n2 + m1 * m2
    hx = np.vstack([x_rows, np.zeros((z_rows.shape[0], n), dtype=np.uint8)])
    hz = np.vstack([np.zeros((x_rows.shape[0], n), dtype=np.uint8), z_rows])
    return hx.astype(np.uint8), hz.astype(np.uint8)


def planar(L: int) -> StabilizerCode:
    """Unrotated planar surface code [[2L^2-2L+1, 1, L]] (section II-A, Fig. 1)."""
    if L < 2:
        raise ValueError("planar code needs L >= 2")
    h = repetition_open(L)
    hx, hz = hypergraph_product(h, h)
    return _finish(f"planar_d{L}", hx, hz, _repetition_product_coords(L, L - 1, L, L - 1))


def toric(L: int) -> StabilizerCode:
    """Toric code [[2L^2, 2, L]] (section II-A); all M = 2L^2 checks kept, two dependent."""
    if L < 2:
        raise ValueError("toric code needs L >= 2")
    h = repetition_cyclic(L)
    hx, hz = hypergraph_product(h, h)
    return _finish(f"toric_L{L}", hx, hz, _repetition_product_coords(L, L, L, L))


def xzzx(L: int) -> StabilizerCode:
    """XZZX surface code on an L x L torus (section II-A).

    Qubit (a, b) has index a*L + b.  The stabilizer of face (a, b) is
    X on (a, b), Z on (a+1, b), Z on (a, b+1), X on (a+1, b+1), indices mod L.
    """
    if L < 3:
        raise ValueError("xzzx code needs L >= 3")
    n = L * L
    hx = np.zeros((n, n), dtype=np.uint8)
    hz = np.zeros((n, n), dtype=np.uint8)

    def q(a, b):
        return (a % L) * L + (b % L)

    for a in range(L):
        for b in range(L):
            r = q(a, b)
            hx[r, q(a, b)] = 1
            hz[r, q(a + 1, b)] = 1
            hz[r, q(a, b + 1)] = 1
            hx[r, q(a + 1, b + 1)] = 1
    a, b = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    return _finish(f"xzzx_L{L}", hx, hz, np.stack([a.ravel(), b.ravel()], axis=1))


def trapping_ring() -> StabilizerCode:
    """Isolated 4-qubit ring of the smallest surface-code trapping set (section II-B2).

    Checks c_k = Z_{q_{k-1}} Z_{q_k} (indices mod 4): c1 = {q4, q1}, c2 = {q1, q2},
    c3 = {q2, q3}, c4 = {q3, q4}.  X errors on q1, q2 give the syndrome [1, 0, 1, 0]
    of section IV-A.
    """
    hz = np.zeros((4, 4), dtype=np.uint8)
    for k in range(4):
        hz[k, (k - 1) % 4] = 1
        hz[k, k] = 1
    hx = np.zeros_like(hz)
    return _finish("trapping_ring", hx, hz)


def _cyclic_shift(k: int) -> np.ndarray:
    s = np.zeros((k, k), dtype=np.uint8)
    for i in range(k):
        s[i, (i + 1) % k] = 1
    return s


def bivariate_bicycle(l: int, m: int, a_terms, b_terms, name: str = None) -> StabilizerCode:
    """Bivariate bicycle code (Bravyi et al. 2024; section IV-C cites it).

    x = S_l (x) I_m and y = I_l (x) S_m generate commuting permutation matrices
    (S_k the k x k cyclic shift); A and B are sums of three monomials, each term a
    pair (i, j) meaning x^i y^j.  X checks [A | B], Z checks [B^T | A^T] on 2lm
    qubits (A and B commute, so the two kinds of checks commute)."""
    x = np.kron(_cyclic_shift(l), np.eye(m, dtype=np.uint8))
    y = np.kron(np.eye(l, dtype=np.uint8), _cyclic_shift(m))

    def poly(terms):
        acc = np.zeros((l * m, l * m), dtype=np.int64)
        for i, j in terms:
            acc += np.linalg.matrix_power(x.astype(np.int64), i) @ np.linalg.matrix_power(y.astype(np.int64), j)
        return (acc & 1).astype(np.uint8)

    A, B = poly(a_terms), poly(b_terms)
    q = l * m
    x_rows = np.hstack([A, B])
    z_rows = np.hstack([B.T, A.T])
    hx = np.vstack([x_rows, np.zeros((q, 2 * q), dtype=np.uint8)])
    hz = np.vstack([np.zeros((q, 2 * q), dtype=np.uint8), z_rows])
    return _finish(name or f"bb_{l}x{m}", hx, hz)


# The published instances [[n, k, d]] -> (l, m, A, B) with A, B as (x power, y power) terms.
BB_CODES = {
    72: (6, 6, [(3, 0), (0, 1), (0, 2)], [(0, 3), (1, 0), (2, 0)]),      # [[72, 12, 6]]
    90: (15, 3, [(9, 0), (0, 1), (0, 2)], [(0, 0), (2, 0), (7, 0)]),     # [[90, 8, 10]]
    108: (9, 6, [(3, 0), (0, 1), (0, 2)], [(0, 3), (1, 0), (2, 0)]),     # [[108, 8, 10]]
    144: (12, 6, [(3, 0), (0, 1), (0, 2)], [(0, 3), (1, 0), (2, 0)]),    # [[144, 12, 12]]
    288: (12, 12, [(3, 0), (0, 2), (0, 7)], [(0, 3), (1, 0), (2, 0)]),   # [[288, 12, 18]]
}


def bb(n: int) -> StabilizerCode:
    l, m, a_terms, b_terms = BB_CODES[n]
    return bivariate_bicycle(l, m, a_terms, b_terms, name=f"bb_n{n}")


def chamon(d: int) -> StabilizerCode:
    """3D Chamon code (Bravyi, Leemhuis, Terhal 2011; section IV-C) on the periodic
    (2d)^3 cubic lattice: qubits on the sites with even coordinate sum, one check per
    odd site v acting as X on v +- e_x, Y on v +- e_y and Z on v +- e_z."""
    if d < 1:
        raise ValueError("chamon code needs d >= 1")
    L = 2 * d
    sites = [(a, b, c) for a in range(L) for b in range(L) for c in range(L)]
    qubits = [s for s in sites if sum(s) % 2 == 0]
    checks = [s for s in sites if sum(s) % 2 == 1]
    qi = {s: i for i, s in enumerate(qubits)}
    n, m = len(qubits), len(checks)
    hx = np.zeros((m, n), dtype=np.uint8)
    hz = np.zeros((m, n), dtype=np.uint8)
    for r, (a, b, c) in enumerate(checks):
        for da in (-1, 1):
            v = qi[((a + da) % L, b, c)]
            hx[r, v] = 1                              # X
        for db in (-1, 1):
            v = qi[(a, (b + db) % L, c)]
            hx[r, v] = 1                              # Y = X and Z
            hz[r, v] = 1
        for dc in (-1, 1):
            v = qi[(a, b, (c + dc) % L)]
            hz[r, v] = 1                              # Z
    return _finish(f"chamon_d{d}", hx, hz)


FAMILIES = {"planar": planar, "toric": toric, "xzzx": xzzx, "bb": bb, "chamon": chamon}


def make(family: str, size: int) -> StabilizerCode:
    return FAMILIES[family](size)


# ---------------------------------------------------------------------------
# Logical operators (section II-A: elements of N(S) \ S)
# ---------------------------------------------------------------------------

def logical_basis(hx: np.ndarray, hz: np.ndarray):
    """Symplectic basis {X_1..X_k, Z_1..Z_k} of N(S) modulo S.

    N(S) is the null space of the symplectic form against the rows of (hx|hz).
    Symplectic Gram-Schmidt on a basis of N(S) pairs up vectors with product 1;
    vectors left without a partner span the radical, which inside N(S) is S
    itself.  The Gram-Schmidt steps act on the basis and on its symplectic Gram
    matrix together.  Returns (lx, lz) with rows ordered X_1..X_k then Z_1..Z_k,
    so that <X_i, Z_j> = delta_ij and all other pairs commute.
    """
    hx = np.asarray(hx, dtype=np.uint8)
    hz = np.asarray(hz, dtype=np.uint8)
    n = hx.shape[1]
    # v = (vx | vz) commutes with every row iff hx.vz + hz.vx = 0.
    b = gf2_nullspace(np.hstack([hz, hx])).astype(np.uint8)
    bf = b.astype(np.float64)
    g = (bf[:, :n] @ bf[:, n:].T + bf[:, n:] @ bf[:, :n].T)
    g = (np.rint(g).astype(np.int64) & 1).astype(np.uint8)
    alive = np.ones(b.shape[0], dtype=bool)
    xs, zs = [], []
    for i in range(b.shape[0]):
        if not alive[i]:
            continue
        cand = np.nonzero(g[i] & alive)[0]
        alive[i] = False
        if cand.size == 0:
            continue  # radical vector: a stabilizer
        j = int(cand[0])
        alive[j] = False
        v, w = b[i].copy(), b[j].copy()
        gv, gw = g[i].copy(), g[j].copy()   # products of every vector with v and with w
        # u <- u + <u,w> v + <u,v> w makes u orthogonal to both v and w.
        cw = gw.astype(bool) & alive
        cv = gv.astype(bool) & alive
        b[cw] ^= v
        b[cv] ^= w
        g[cw] ^= g[i]
        g[cv] ^= g[j]
        g[:, cw] ^= g[:, [i]]
        g[:, cv] ^= g[:, [j]]
        xs.append(v)
        zs.append(w)
    k = len(xs)
    if k == 0:
        return np.zeros((0, n), np.uint8), np.zeros((0, n), np.uint8)
    basis = np.array(xs + zs, dtype=np.uint8)
    return basis[:, :n].copy(), basis[:, n:].copy()


# ---------------------------------------------------------------------------
# Noise and priors (section IV: depolarizing channel, X/Y/Z each p/3)
# ---------------------------------------------------------------------------

def depolarizing_probs(n: int, p: float) -> np.ndarray:
    """Per-qubit (p_X, p_Y, p_Z) for the depolarizing channel, float64 (n, 3)."""
    return np.tile(np.array([p / 3.0, p / 3.0, p / 3.0]), (n, 1))


def biased_probs(n: int, p: float, fz: float = 2.0 / 3.0, fx: float = 1.0 / 6.0,
                 fy: float = 1.0 / 6.0) -> np.ndarray:
    """Per-qubit (p_X, p_Y, p_Z) for biased noise with fractions of p (section IV-B3)."""
    return np.tile(np.array([fx * p, fy * p, fz * p]), (n, 1))


def thresholds(px: float, py: float, pz: float) -> np.ndarray:
    """Integer Pauli thresholds of 2^32 for the sampler: t_W = round(p_W * 2^32).

    A uniform 32-bit word u picks X if u < tX, Y if u < tX+tY, Z if
    u < tX+tY+tZ, else I.
    """
    t = np.array([round(px * 2 ** 32), round(py * 2 ** 32), round(pz * 2 ** 32)], dtype=np.uint64)
    if int(t.sum()) >= 2 ** 32:
        raise ValueError("total error probability must be below 1")
    return t.astype(np.uint32)


def config_seed(config: int, code_index: int, p_index: int) -> int:
    """64-bit sampler key used for a benchmark configuration, code and error rate."""
    return 24071152300 + 10000 * config + 100 * code_index + p_index
