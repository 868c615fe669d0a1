"""Exact logical error rates on the distance-3 planar code by full enumeration.

Writes ``d3_exact_ler.json`` beside this file.  Uses only the FP64 oracle and
the code generator: every one of the 2^12 syndromes is decoded once; the
probability of each of its four cosets (reference error x logical class x all
2^12 stabilizers) is summed exactly under the depolarizing channel (X, Y, Z
each p/3, section IV).  A decoder fails on syndrome s unless it converges to
an estimate in the coset that actually occurred, so its exact
logical error rate is 1 - sum_s [converged] P(coset of the estimate); the
maximum-likelihood decoder of eq. qecobject picks the heaviest coset and
gives a lower bound for every decoder.

Run: python -m tests.golden.make_d3_exact
"""
import json
import os

import numpy as np

import qecgen
from oracle import oracle as O

P_CONFIG = 0.05
CASES = [("bp", 1.0), ("ewainit", 0.5)]


def _solve_unit_syndromes(code):
    """For each check c a Pauli (x|z bits) whose syndrome is the unit vector e_c."""
    m, n = code.m, code.n
    A = np.hstack([code.hz, code.hx]).astype(np.uint8)   # syndrome of (ex | ez)
    out = []
    for c in range(m):
        aug = np.hstack([A, (np.arange(m) == c).astype(np.uint8)[:, None]])
        rows, cols = aug.shape
        r, piv = 0, []
        for col in range(cols - 1):
            nz = np.nonzero(aug[r:, col])[0]
            if nz.size == 0:
                continue
            p = r + nz[0]
            aug[[r, p]] = aug[[p, r]]
            for i in range(rows):
                if i != r and aug[i, col]:
                    aug[i] ^= aug[r]
            piv.append(col)
            r += 1
            if r == rows:
                break
        x = np.zeros(2 * n, np.uint8)
        for i, col in enumerate(piv):
            x[col] = aug[i, -1]
        assert np.array_equal((A.astype(int) @ x) % 2, (np.arange(m) == c).astype(int))
        out.append(x)
    return np.array(out)


def _mask(bits):
    return int(sum(int(b) << i for i, b in enumerate(bits)))


def exact_ler(variant, alpha, p=P_CONFIG, max_iter=50):
    code = qecgen.planar(3)
    n, m = code.n, code.m
    assert code.rank == m
    unit = _solve_unit_syndromes(code)
    ux = np.array([_mask(u[:n]) for u in unit])
    uz = np.array([_mask(u[n:]) for u in unit])
    gx = np.array([_mask(r) for r in code.hx])
    gz = np.array([_mask(r) for r in code.hz])
    idx = np.arange(2 ** m)
    bits = (idx[:, None] >> np.arange(m)) & 1
    sx = np.bitwise_xor.reduce(np.where(bits, gx[None], 0), axis=1)
    sz = np.bitwise_xor.reduce(np.where(bits, gz[None], 0), axis=1)
    lx0, lz0 = _mask(code.lx[0]), _mask(code.lz[0])
    lx1, lz1 = _mask(code.lx[1]), _mask(code.lz[1])
    log_x = [0, lx0, lx1, lx0 ^ lx1]
    log_z = [0, lz0, lz1, lz0 ^ lz1]
    pop = np.array([bin(i).count("1") for i in range(2 ** n)])
    wprob = (1 - p) ** (n - np.arange(n + 1)) * (p / 3) ** np.arange(n + 1)

    def sp(ax, az, bx, bz):
        return (bin(ax & bz).count("1") + bin(az & bx).count("1")) & 1

    def cls(rx, rz):
        return (sp(rx, rz, lx0, lz0), sp(rx, rz, lx1, lz1))

    classes = [cls(log_x[k], log_z[k]) for k in range(4)]
    # decode every syndrome once
    synd = bits.astype(np.uint8)
    pi = O.prior_llr(qecgen.depolarizing_probs(n, p))
    r = O.decode(code.hx, code.hz, O.Params(variant=variant, alpha=alpha, max_iter=max_iter), pi, synd)
    success = 0.0
    ml_success = 0.0
    for s in range(2 ** m):
        bx = int(np.bitwise_xor.reduce(np.where(bits[s], ux, 0)))
        bz = int(np.bitwise_xor.reduce(np.where(bits[s], uz, 0)))
        pc = []
        for k in range(4):
            w = pop[(sx ^ bx ^ log_x[k]) | (sz ^ bz ^ log_z[k])]
            pc.append(float(wprob[w].sum()))
        ml_success += max(pc)
        if r["conv"][s]:
            est = r["est"][s]
            ex, ez = _mask(est & 1), _mask(est >> 1)
            k = classes.index(cls(ex ^ bx, ez ^ bz))
            success += pc[k]
    return 1.0 - success, 1.0 - ml_success


def main():
    O.build()
    out = {"_cite": "planar d=3, depolarizing p=0.05, iter_max 50 (sections II-B1, III-B, IV); "
                    "written by tests/golden/make_d3_exact.py from the FP64 oracle",
           "p": P_CONFIG, "max_iter": 50}
    ml = None
    for variant, alpha in CASES:
        e, ml = exact_ler(variant, alpha)
        out[f"{variant}_a{alpha}"] = {"exact_ler": e}
    out["ml_ler"] = ml
    with open(os.path.join(os.path.dirname(__file__), "d3_exact_ler.json"), "w") as f:
        json.dump(out, f, indent=2)
    print(json.dumps(out, indent=2))


if __name__ == "__main__":
    main()
