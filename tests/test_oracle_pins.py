"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a library
routine (numpy's Philox), high-precision evaluation of the paper's literal
formulas (mpmath), brute-force exact marginals on cycle-free Tanner graphs,
an independent probability-domain quaternary BP, the paper's closed forms
(Theorem 1, Appendix B) and special cases (alpha = 1), symmetry invariants,
exhaustive small-code decoding and an exact enumeration of every syndrome of
the distance-3 planar code.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import qecgen
from oracle import oracle as O
from qecgen import symplectic_product

GOLD = os.path.join(os.path.dirname(__file__), "golden")

# Pauli codes: bit0 = x, bit1 = z.  COMM[a][b] = 1 iff a and b anticommute.
COMM = np.array([[((a & 1) & (b >> 1)) ^ ((a >> 1) & (b & 1)) for b in range(4)] for a in range(4)])
XYZ = (1, 3, 2)   # Pauli codes in the LLR triple order (X, Y, Z)


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


def syndrome_np(hx, hz, err):
    err = np.atleast_2d(err)
    return symplectic_product(hx, hz, err & 1, err >> 1).T.astype(np.uint8)


def clifford_relabel(code, rng):
    """Apply an independent random permutation of (X, Y, Z) to every qubit's column."""
    lab = code.labels()
    perms = [rng.permutation([1, 2, 3]) for _ in range(code.n)]
    new = np.zeros_like(lab)
    for v in range(code.n):
        mp = {0: 0, 1: perms[v][0], 2: perms[v][1], 3: perms[v][2]}
        new[:, v] = [mp[int(x)] for x in lab[:, v]]
    return (new & 1).astype(np.uint8), (new >> 1).astype(np.uint8), perms


# ---------------------------------------------------------------------------
# Sampler
# ---------------------------------------------------------------------------

def test_philox_matches_numpy():
    # numpy.random.Philox is Philox4x64-10; its k-th block is the bijection at counter c + k + 1.
    rng = np.random.default_rng(7)
    for _ in range(20):
        key = rng.integers(0, 2 ** 63, size=2, dtype=np.uint64)
        ctr = rng.integers(0, 2 ** 63, size=4, dtype=np.uint64)
        bg = np.random.Philox(key=key, counter=ctr)
        want = bg.random_raw(4).astype(np.uint64)
        c1 = ctr.copy()
        c1[0] += np.uint64(1)
        assert np.array_equal(O.philox4x64_10(c1, key), want)


def test_sampler_frequencies_and_syndromes():
    code = qecgen.toric(4)
    p = np.array([0.02, 0.05, 0.11])  # X, Y, Z
    thr = qecgen.thresholds(*p)
    err, syn = O.sample(code.hx, code.hz, 20000, thr, seed=99, stream=3)
    n_tot = err.size
    for pauli, pw in zip((1, 3, 2), p):
        k = int((err == pauli).sum())
        lo, hi = O.wilson_ci(k, n_tot, z=4.0)
        assert lo <= pw <= hi
    # syndrome is <H, E> mod 2, independently evaluated
    assert np.array_equal(syn, syndrome_np(code.hx, code.hz, err))
    # shot0 offsets the counter: shots 10.. of a run equal shots 0.. of an offset run
    e2, s2 = O.sample(code.hx, code.hz, 50, thr, seed=99, stream=3, shot0=10)
    assert np.array_equal(e2, err[10:60]) and np.array_equal(s2, syn[10:60])
    # a different stream changes the draw
    e3, _ = O.sample(code.hx, code.hz, 50, thr, seed=99, stream=4)
    assert not np.array_equal(e3, err[:50])


def test_syndrome_linearity_and_stabilizers():
    code = qecgen.planar(5)
    rng = np.random.default_rng(3)
    thr = qecgen.thresholds(0.05, 0.05, 0.05)
    err, syn = O.sample(code.hx, code.hz, 64, thr, seed=5)
    # s(E1 E2) = s(E1) + s(E2); stabilizer rows have zero syndrome
    a, b = err[:32], err[32:]
    assert np.array_equal(syndrome_np(code.hx, code.hz, a ^ b), syn[:32] ^ syn[32:])
    stab = code.labels()
    assert not syndrome_np(code.hx, code.hz, stab).any()
    # multiplying errors by random stabilizers keeps the syndrome
    mult = stab[rng.integers(0, code.m, size=32)]
    assert np.array_equal(syndrome_np(code.hx, code.hz, a ^ mult), syn[:32])


# ---------------------------------------------------------------------------
# Elementary functions against the paper's literal formulas at 60 digits
# ---------------------------------------------------------------------------

def test_lambda_matches_literal_formula():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 60
    rng = np.random.default_rng(11)
    for _ in range(400):
        L = rng.uniform(-40, 40, size=3)
        H = int(rng.choice([1, 2, 3]))
        LH = L[XYZ.index(H)]
        e = [mpmath.exp(-mpmath.mpf(float(x))) for x in L]
        want = mpmath.log((1 + mpmath.exp(-mpmath.mpf(float(LH)))) / (e[0] + e[1] + e[2] - mpmath.exp(-mpmath.mpf(float(LH)))))
        got = O.lam(H, L)
        assert abs(got - float(want)) <= 1e-13 * max(1.0, abs(float(want)))


def test_check_rule_matches_tanh_product():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 80
    rng = np.random.default_rng(12)
    for _ in range(400):
        d = int(rng.integers(1, 4))
        ms = rng.uniform(-30, 30, size=d) * (10.0 ** rng.uniform(-3, 0, size=d))
        prod = mpmath.mpf(1)
        for x in ms:
            prod *= mpmath.tanh(mpmath.mpf(float(x)) / 2)
        want = float(2 * mpmath.atanh(prod))
        sgn = -1.0 if (ms < 0).sum() % 2 else 1.0
        got = sgn * O.phi(sum(O.phi(abs(x)) for x in ms))
        assert abs(got - want) <= 1e-12 * max(1.0, abs(want))
    assert O.phi(0.0) == math.inf and O.phi(math.inf) == 0.0


# ---------------------------------------------------------------------------
# Exact marginals on cycle-free Tanner graphs (BP is exact on trees)
# ---------------------------------------------------------------------------

def random_forest(n, m, rng):
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            a = parent[a]
        return a

    rows = []
    for _ in range(1000):
        if len(rows) == m:
            break
        d = int(rng.integers(2, 4))
        vs = rng.choice(n, size=d, replace=False)
        roots = [find(int(v)) for v in vs]
        if len(set(roots)) < d:
            continue
        for r in roots[1:]:
            parent[r] = roots[0]
        rows.append((vs, rng.integers(1, 4, size=d)))
    hx = np.zeros((len(rows), n), np.uint8)
    hz = np.zeros_like(hx)
    for i, (vs, ls) in enumerate(rows):
        for v, l in zip(vs, ls):
            hx[i, v] = l & 1
            hz[i, v] = l >> 1
    return hx, hz


def brute_force_llr(hx, hz, probs, s):
    n = hx.shape[1]
    allE = np.array(list(itertools.product(range(4), repeat=n)), dtype=np.uint8)
    S = syndrome_np(hx, hz, allE)
    pfull = np.column_stack([1 - probs.sum(1), probs[:, 0], probs[:, 2], probs[:, 1]])
    P = np.ones(len(allE))
    for v in range(n):
        P *= pfull[v, allE[:, v]]
    mask = np.all(S == s, axis=1)
    Q = np.zeros((n, 3))
    for v in range(n):
        marg = [P[mask & (allE[:, v] == c)].sum() for c in (0, 1, 3, 2)]
        Q[v] = np.log(marg[0]) - np.log(marg[1:])
    return Q, allE, P


@pytest.mark.parametrize("seed", range(12))
def test_tree_exact_marginals(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(4, 8))
    hx, hz = random_forest(n, int(rng.integers(2, n)), rng)
    m = hx.shape[0]
    probs = rng.dirichlet([8, 1, 1, 1], size=n)[:, 1:]
    pi = O.prior_llr(probs)
    # a syndrome drawn from the prior
    allE = np.array(list(itertools.product(range(4), repeat=n)), dtype=np.uint8)
    pfull = np.column_stack([1 - probs.sum(1), probs[:, 0], probs[:, 2], probs[:, 1]])
    P = np.prod(pfull[np.arange(n), allE], axis=1)
    e0 = allE[rng.choice(len(allE), p=P / P.sum())]
    s = syndrome_np(hx, hz, e0)[0]
    Qb, _, _ = brute_force_llr(hx, hz, probs, s)
    r = O.decode(hx, hz, O.Params(variant="bp", max_iter=2 * (n + m), stop_on_syndrome=False,
                                  clamp=math.inf), pi, s[None], want_q=True)
    assert np.allclose(r["q"][0], Qb, rtol=1e-10, atol=1e-10)


# ---------------------------------------------------------------------------
# Independent probability-domain quaternary BP on graphs with cycles
# ---------------------------------------------------------------------------

def prob_bp4(hx, hz, probs, s, T, variant="bp", alpha=1.0):
    """Quaternary sum-product with 4-vector messages (I, X, Z, Y by Pauli code).

    Check messages sum explicitly over every Pauli configuration of the other
    neighbours.  EWAInit's prior update is the geometric mixture
    p^{(t)} ~ p0^alpha * post^{(t-1)}^(1-alpha); Momentum (gamma = 0) mixes the
    BP posterior with the previous one the same way, and its outgoing message
    divides the check's own incoming message out of that posterior.
    Returns Q^{(t)} (LLR form) for t = 1..T.
    """
    m, n = hx.shape
    lab = (hx | (hz << 1)).astype(int)
    edges = [(c, v) for c in range(m) for v in range(n) if lab[c, v]]
    p0 = np.column_stack([1 - probs.sum(1), probs[:, 0], probs[:, 2], probs[:, 1]])
    q = {e: p0[e[1]].copy() for e in edges}
    post_prev = p0.copy()
    prior = p0.copy()
    out = []
    for t in range(1, T + 1):
        if variant == "ewainit" and t > 1:
            prior = p0 ** alpha * post_prev ** (1 - alpha)
            prior /= prior.sum(1, keepdims=True)
        r = {}
        for (c, v) in edges:
            others = [u for u in range(n) if lab[c, u] and u != v]
            rv = np.zeros(4)
            for P in range(4):
                tot = 0.0
                for conf in itertools.product(range(4), repeat=len(others)):
                    par = COMM[lab[c, v], P]
                    w = 1.0
                    for u, Pu in zip(others, conf):
                        par ^= COMM[lab[c, u], Pu]
                        w *= q[(c, u)][Pu]
                    if par == s[c]:
                        tot += w
                rv[P] = tot
            r[(c, v)] = rv / rv.sum()
        base = p0 if variant in ("bp", "momentum") else prior
        post = base.copy()
        for (c, v) in edges:
            post[v] = post[v] * r[(c, v)]
        post /= post.sum(1, keepdims=True)
        if variant == "momentum":
            post = post ** alpha * post_prev ** (1 - alpha)
            post /= post.sum(1, keepdims=True)
        for (c, v) in edges:
            if variant == "momentum":
                qq = post[v] / r[(c, v)]
            else:
                qq = base[v].copy()
                for (c2, v2) in edges:
                    if v2 == v and c2 != c:
                        qq = qq * r[(c2, v2)]
            q[(c, v)] = qq / qq.sum()
        post_prev = post
        out.append(np.log(post[:, [0]]) - np.log(post[:, [1, 3, 2]]))
    return np.array(out)


@pytest.mark.parametrize("make", [lambda: qecgen.planar(3), lambda: qecgen.toric(3),
                                  lambda: qecgen.xzzx(3)])
@pytest.mark.parametrize("variant,alpha", [("bp", 1.0), ("ewainit", 0.6), ("momentum", 0.7)])
def test_probability_domain_bp4(make, variant, alpha):
    code = make()
    rng = np.random.default_rng(5)
    hx, hz, _ = clifford_relabel(code, rng)      # puts Y labels on the edges too
    probs = rng.uniform(0.005, 0.04, size=(code.n, 3))
    e = np.zeros(code.n, np.uint8)
    e[rng.choice(code.n, 2, replace=False)] = rng.integers(1, 4, size=2)
    s = syndrome_np(hx, hz, e)[0]
    T = 6
    want = prob_bp4(hx, hz, probs, s, T, variant, alpha)
    r = O.decode(hx, hz, O.Params(variant=variant, max_iter=T, stop_on_syndrome=False,
                                  clamp=math.inf, alpha=alpha), O.prior_llr(probs), s[None],
                 want_trace=True)
    assert np.allclose(r["q_trace"][0], want, rtol=1e-9, atol=1e-9)


# ---------------------------------------------------------------------------
# Special cases and closed forms (sections III-A1, III-B, Appendix B)
# ---------------------------------------------------------------------------

def _toric_batch(shots=64, p=0.08, seed=21):
    code = qecgen.toric(5)
    thr = qecgen.thresholds(p / 3, p / 3, p / 3)
    err, syn = O.sample(code.hx, code.hz, shots, thr, seed=seed)
    pi = O.prior_llr(qecgen.depolarizing_probs(code.n, p))
    return code, err, syn, pi


def test_ewainit_alpha_one_is_bp_bit_exact():
    code, _, syn, pi = _toric_batch()
    a = O.decode(code.hx, code.hz, O.Params(variant="bp", max_iter=40), pi, syn, want_q=True, want_msgs=True)
    b = O.decode(code.hx, code.hz, O.Params(variant="ewainit", alpha=1.0, max_iter=40), pi, syn,
                 want_q=True, want_msgs=True)
    for k in ("est", "conv", "iters", "q", "mvc", "mcv"):
        assert np.array_equal(a[k], b[k]), k


def test_momentum_alpha_one_gamma_zero_is_bp():
    code, _, syn, pi = _toric_batch()
    a = O.decode(code.hx, code.hz, O.Params(variant="bp", max_iter=12, stop_on_syndrome=False),
                 pi, syn, want_trace=True)
    b = O.decode(code.hx, code.hz, O.Params(variant="momentum", alpha=1.0, gamma=0.0, max_iter=12,
                                            stop_on_syndrome=False), pi, syn, want_trace=True)
    assert np.allclose(a["q_trace"], b["q_trace"], rtol=1e-12, atol=1e-11)


@pytest.mark.parametrize("alpha", [0.3, 0.7])
def test_theorem1_ewainit_closed_form(alpha):
    # Q^{(t)} = Pi^{(0)} + sum_{k=0}^{t-1} (1-alpha)^k M^{(t-k)}   (Theorem 1, k up to t-1)
    code, _, syn, pi = _toric_batch(shots=16)
    T = 10
    r = O.decode(code.hx, code.hz, O.Params(variant="ewainit", alpha=alpha, max_iter=T,
                                            stop_on_syndrome=False), pi, syn, want_trace=True)
    Qt, Mt = r["q_trace"], r["m_trace"]
    for t in range(1, T + 1):
        want = pi[None] + sum((1 - alpha) ** k * Mt[:, t - k - 1] for k in range(t))
        assert np.allclose(Qt[:, t - 1], want, rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("alpha", [0.4, 0.8])
def test_momentum_closed_form_gamma_zero(alpha):
    # Appendix B: Q^{(t)} = Pi^{(0)} + sum_{k=0}^{t-1} alpha (1-alpha)^k M^{(t-k)}
    code, _, syn, pi = _toric_batch(shots=16)
    T = 10
    r = O.decode(code.hx, code.hz, O.Params(variant="momentum", alpha=alpha, gamma=0.0, max_iter=T,
                                            stop_on_syndrome=False), pi, syn, want_trace=True)
    Qt, Mt = r["q_trace"], r["m_trace"]
    for t in range(1, T + 1):
        want = pi[None] + sum(alpha * (1 - alpha) ** k * Mt[:, t - k - 1] for k in range(t))
        assert np.allclose(Qt[:, t - 1], want, rtol=1e-12, atol=1e-10)


def test_momentum_alpha_one_identity():
    # eq. mombp3-4 with alpha = 1: Q^{(t)} = gamma (Q^{(t-1)} - g^{(t-1)}) + (1-gamma)(Pi + M^{(t)}),
    # where with alpha = 1 the momentum is g^{(t)} = Q^{(t-1)} - Q^{(t)}.
    code, _, syn, pi = _toric_batch(shots=16)
    g_ = 0.35
    T = 8
    r = O.decode(code.hx, code.hz, O.Params(variant="momentum", alpha=1.0, gamma=g_, max_iter=T,
                                            stop_on_syndrome=False), pi, syn, want_trace=True)
    Q = np.concatenate([np.broadcast_to(pi, (16, 1) + pi.shape), r["q_trace"]], axis=1)
    g = np.zeros_like(Q)
    for t in range(1, T + 1):
        g[:, t] = Q[:, t - 1] - Q[:, t]
    for t in range(2, T + 1):
        want = g_ * (Q[:, t - 1] - g[:, t - 1]) + (1 - g_) * (pi[None] + r["m_trace"][:, t - 1])
        assert np.allclose(Q[:, t], want, rtol=1e-11, atol=1e-10)


def test_adagrad_step_invariants():
    # eq. boost: each adaptive step has magnitude alpha |g'| / (sqrt(G) + eps) <= alpha, and the
    # first adaptive step (t = 2, G = g'^2) is alpha |g'| / (|g'| + eps), for every gradient.
    code, _, syn, pi = _toric_batch(shots=16)
    T, a = 10, 5.0
    r = O.decode(code.hx, code.hz, O.Params(variant="adagrad", alpha=a, max_iter=T,
                                            stop_on_syndrome=False), pi, syn, want_trace=True)
    Q, M = r["q_trace"], r["m_trace"]
    assert np.allclose(Q[:, 0], pi[None] + M[:, 0], rtol=1e-14, atol=1e-12)   # t = 1 is plain BP
    steps = np.abs(np.diff(Q, axis=1))
    assert np.all(steps <= a * (1 + 1e-12))
    gp = M[:, 0] - M[:, 1]          # Q^{(1)} - Pi - M^{(2)} with Q^{(1)} = Pi + M^{(1)}
    assert (np.abs(gp) > 1e-3).mean() > 0.3
    step = np.abs(Q[:, 1] - Q[:, 0])
    assert np.allclose(step, a * np.abs(gp) / (np.abs(gp) + 1e-8), rtol=1e-9, atol=1e-9)
    # a gradient that vanishes gives no step, bit for bit
    assert np.all(step[gp == 0] == 0)
    # accumulating G from t = 1 gives a smaller first adaptive step
    r2 = O.decode(code.hx, code.hz, O.Params(variant="adagrad", alpha=a, max_iter=T, stop_on_syndrome=False,
                                             adagrad_g_from_t1=True), pi, syn, want_trace=True)
    s2 = np.abs(r2["q_trace"][:, 1] - r2["q_trace"][:, 0])
    assert np.all(s2 <= np.abs(Q[:, 1] - Q[:, 0]) + 1e-12)


def test_adagrad_steps_at_rounding_level_gradients_mpmath():
    """Eq. boost has no threshold: wherever the first adaptive gradient g' = D^{(1)} - M^{(2)}
    (D^{(1)} = M^{(1)}) is not exactly 0, the oracle moves Q by alpha |g'| / (|g'| + eps), also
    where g' is FP64 rounding residue (1e-16 .. 1e-15, a step of about 5e-8 .. 4e-7), and
    only where it is exactly 0 does Q stay put.  g' and the prescribed step are evaluated in
    60-digit mpmath from the oracle's traced message sums."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 60
    code = qecgen.planar(3)
    probs = qecgen.depolarizing_probs(code.n, 0.08)
    _, syn = O.sample(code.hx, code.hz, 2000, qecgen.thresholds(*probs[0]), seed=5)
    pi = O.prior_llr(probs)
    a, eps = 5.0, 1e-8
    r = O.decode(code.hx, code.hz, O.Params(variant="adagrad", alpha=a, eps=eps, max_iter=3, stop_on_syndrome=False),
                 pi, syn, want_trace=True)
    Q, M = r["q_trace"], r["m_trace"]
    step = (Q[:, 1] - Q[:, 0]).ravel()
    m1, m2 = M[:, 0].ravel(), M[:, 1].ravel()
    tiny = 0
    for i in range(m1.size):
        g = mp.mpf(float(m1[i])) - mp.mpf(float(m2[i]))
        if g == 0:
            assert step[i] == 0.0, i
            continue
        want = -a * g / (abs(g) + mp.mpf(eps))   # Q^{(2)} - Q^{(1)} = D^{(2)} - D^{(1)}
        # Q is traced as Pi + D rounded, so the difference carries ~1e-15 absolute rounding
        assert abs(mp.mpf(float(step[i])) - want) <= mp.mpf("1e-6") * abs(want) + mp.mpf("4e-15"), (i, g, step[i])
        if abs(g) < mp.mpf("1e-12"):
            tiny += 1
            assert step[i] != 0.0 and abs(step[i]) > 1e-9, (i, g, step[i])
    assert tiny >= 10, tiny


def prob_bp4_optim(hx, hz, probs, s, T, variant, alpha, gamma=0.0, eps=1e-8, g_from_t1=False):
    """Probability-domain quaternary BP whose posterior follows a library optimiser.

    Check messages are the explicit sums over neighbour configurations of
    ``prob_bp4``.  M_{v,W} = sum_c ln(r_{c->v}(I) / r_{c->v}(W)) is the LLR form of
    the product of the incoming check messages.  Momentum-BP (eqs. mombp1-3) and
    AdaGrad-BP (eq. boost) treat Q - Pi - M as the gradient of the posterior; here
    torch.optim.SGD (heavy ball with dampening gamma, i.e. g = gamma g + (1 - gamma)
    grad, Q -= alpha g, momentum buffer starting at 0) and torch.optim.Adagrad
    (G += grad^2, Q -= alpha grad / (sqrt(G) + eps)) take that step.  AdaGrad's first
    iteration is the plain BP posterior with G = 0 (or G = grad^2 with
    ``g_from_t1``).  The outgoing message divides the check's own incoming
    message out of the posterior (probability form of lambda(Q - m_{c->v})).
    Returns Q^{(t)} for t = 1..T.
    """
    torch = pytest.importorskip("torch")
    m, n = hx.shape
    lab = (hx | (hz << 1)).astype(int)
    edges = [(c, v) for c in range(m) for v in range(n) if lab[c, v]]
    p0 = np.column_stack([1 - probs.sum(1), probs[:, 0], probs[:, 2], probs[:, 1]])
    q = {e: p0[e[1]].copy() for e in edges}
    pi = torch.tensor(np.log(p0[:, [0]]) - np.log(p0[:, [1, 3, 2]]), dtype=torch.float64)
    Q = pi.clone().requires_grad_(True)
    if variant == "momentum":
        opt = torch.optim.SGD([Q], lr=alpha, momentum=gamma, dampening=gamma)
        opt.state[Q]["momentum_buffer"] = torch.zeros_like(Q)
    else:
        opt = torch.optim.Adagrad([Q], lr=alpha, eps=eps, initial_accumulator_value=0.0)
    out = []
    for t in range(1, T + 1):
        r = {}
        for (c, v) in edges:
            others = [u for u in range(n) if lab[c, u] and u != v]
            rv = np.zeros(4)
            for P in range(4):
                tot = 0.0
                for conf in itertools.product(range(4), repeat=len(others)):
                    par = COMM[lab[c, v], P]
                    w = 1.0
                    for u, Pu in zip(others, conf):
                        par ^= COMM[lab[c, u], Pu]
                        w *= q[(c, u)][Pu]
                    if par == s[c]:
                        tot += w
                rv[P] = tot
            r[(c, v)] = rv / rv.sum()
        M = np.zeros((n, 3))
        for (c, v) in edges:
            M[v] += np.log(r[(c, v)][0]) - np.log(r[(c, v)][[1, 3, 2]])
        M = torch.tensor(M)
        with torch.no_grad():
            if variant == "adagrad" and t == 1:
                if g_from_t1:
                    opt.state[Q]["sum"].copy_((Q - pi - M) ** 2)
                Q.copy_(pi + M)
            else:
                Q.grad = (Q - pi - M).detach().clone()
                opt.step()
        Qn = Q.detach().numpy().copy()
        post = np.column_stack([np.ones(n), np.exp(-Qn[:, 0]), np.exp(-Qn[:, 2]), np.exp(-Qn[:, 1])])
        post /= post.sum(1, keepdims=True)
        for (c, v) in edges:
            qq = post[v] / r[(c, v)]
            q[(c, v)] = qq / qq.sum()
        out.append(Qn)
    return np.array(out)


@pytest.mark.parametrize("make", [lambda: qecgen.planar(3), lambda: qecgen.toric(3),
                                  lambda: qecgen.xzzx(3)])
@pytest.mark.parametrize("variant,alpha,gamma,g1", [("momentum", 0.7, 0.3, False), ("momentum", 0.5, 0.7, False),
                                                    ("adagrad", 5.0, 0.0, False), ("adagrad", 1.0, 0.0, False),
                                                    ("adagrad", 5.0, 0.0, True)])
def test_optimiser_posteriors_probability_domain(make, variant, alpha, gamma, g1):
    # Momentum-BP with gamma != 0 and AdaGrad-BP on graphs with cycles, Y labels and
    # non-uniform priors, against probability-domain BP driven by torch's SGD / Adagrad.
    code = make()
    rng = np.random.default_rng(5)
    hx, hz, _ = clifford_relabel(code, rng)
    probs = rng.uniform(0.005, 0.04, size=(code.n, 3))
    e = np.zeros(code.n, np.uint8)
    e[rng.choice(code.n, 2, replace=False)] = rng.integers(1, 4, size=2)
    s = syndrome_np(hx, hz, e)[0]
    T = 8
    want = prob_bp4_optim(hx, hz, probs, s, T, variant, alpha, gamma, g_from_t1=g1)
    r = O.decode(hx, hz, O.Params(variant=variant, max_iter=T, stop_on_syndrome=False, clamp=math.inf,
                                  alpha=alpha, gamma=gamma, adagrad_g_from_t1=g1),
                 O.prior_llr(probs), s[None], want_trace=True)
    assert np.allclose(r["q_trace"][0], want, rtol=1e-11, atol=1e-11)


# ---------------------------------------------------------------------------
# Invariants
# ---------------------------------------------------------------------------

def test_check_node_invariants():
    code = qecgen.planar(5)
    rng = np.random.default_rng(8)
    probs = rng.uniform(0.01, 0.05, size=(code.n, 3))
    pi = O.prior_llr(probs)
    s = rng.integers(0, 2, size=code.m).astype(np.uint8)
    p1 = O.Params(variant="bp", max_iter=2, stop_on_syndrome=False, clamp=math.inf)
    a = O.decode(code.hx, code.hz, p1, pi, s[None], want_msgs=True)
    lab = code.labels()
    edges = [(c, v) for c in range(code.m) for v in range(code.n) if lab[c, v]]
    # flipping s_c negates exactly the outgoing messages of check c
    c0 = 7
    s2 = s.copy()
    s2[c0] ^= 1
    b = O.decode(code.hx, code.hz, O.Params(variant="bp", max_iter=1, stop_on_syndrome=False,
                                            clamp=math.inf), pi, s2[None], want_msgs=True)
    a1 = O.decode(code.hx, code.hz, O.Params(variant="bp", max_iter=1, stop_on_syndrome=False,
                                             clamp=math.inf), pi, s[None], want_msgs=True)
    for k, (c, v) in enumerate(edges):
        if c == c0:
            assert b["mcv"][0, k] == -a1["mcv"][0, k]
        else:
            assert b["mcv"][0, k] == a1["mcv"][0, k]
    # |m_{c->v}| <= min over the other neighbours of |m_{v'->c}| (messages of the previous step)
    prev = a1["mvc"][0]
    cur = a["mcv"][0]
    for k, (c, v) in enumerate(edges):
        others = [j for j, (c2, v2) in enumerate(edges) if c2 == c and v2 != v]
        assert abs(cur[k]) <= min(abs(prev[j]) for j in others) * (1 + 1e-12)


def test_local_clifford_equivariance():
    code = qecgen.planar(5)
    rng = np.random.default_rng(9)
    probs = rng.uniform(0.005, 0.05, size=(code.n, 3))
    thr = qecgen.thresholds(0.03, 0.03, 0.03)
    err, syn = O.sample(code.hx, code.hz, 64, thr, seed=77)
    hx2, hz2, perms = clifford_relabel(code, rng)
    # priors follow the relabelling: new Pauli perm[W] carries the old probability of W
    probs2 = np.zeros_like(probs)
    for v in range(code.n):
        mp = {1: perms[v][0], 2: perms[v][1], 3: perms[v][2]}
        for W_old in (1, 2, 3):
            probs2[v, XYZ.index(mp[W_old])] = probs[v, XYZ.index(W_old)]
    for variant, alpha in (("bp", 1.0), ("ewainit", 0.6), ("momentum", 0.5), ("adagrad", 5.0)):
        prm = O.Params(variant=variant, alpha=alpha, max_iter=30)
        a = O.decode(code.hx, code.hz, prm, O.prior_llr(probs), syn, want_q=True)
        b = O.decode(hx2, hz2, prm, O.prior_llr(probs2), syn, want_q=True)
        assert np.array_equal(a["conv"], b["conv"]) and np.array_equal(a["iters"], b["iters"])
        for v in range(code.n):
            mp = {0: 0, 1: perms[v][0], 2: perms[v][1], 3: perms[v][2]}
            assert np.array_equal(np.vectorize(mp.get)(a["est"][:, v]), b["est"][:, v])
            for W_old in (1, 2, 3):
                assert np.allclose(a["q"][:, v, XYZ.index(W_old)], b["q"][:, v, XYZ.index(mp[W_old])],
                                   rtol=1e-13, atol=1e-12)


def test_qubit_and_check_relabelling():
    code = qecgen.xzzx(5)
    rng = np.random.default_rng(10)
    pq = rng.permutation(code.n)
    pc = rng.permutation(code.m)
    hx2, hz2 = code.hx[pc][:, pq], code.hz[pc][:, pq]
    thr = qecgen.thresholds(0.03, 0.03, 0.03)
    _, syn = O.sample(code.hx, code.hz, 64, thr, seed=78)
    pi = O.prior_llr(rng.uniform(0.005, 0.05, size=(code.n, 3)))
    for variant, alpha in (("bp", 1.0), ("ewainit", 0.5)):
        prm = O.Params(variant=variant, alpha=alpha, max_iter=30)
        a = O.decode(code.hx, code.hz, prm, pi, syn, want_q=True)
        b = O.decode(hx2, hz2, prm, pi[pq], syn[:, pc], want_q=True)
        assert np.array_equal(a["est"][:, pq], b["est"])
        assert np.array_equal(a["iters"], b["iters"])
        assert np.allclose(a["q"][:, pq], b["q"], rtol=1e-12, atol=1e-11)


def test_trapping_ring_symmetry_never_converges():
    # Section IV-A / Table I: on the (4,0) trapping set with syndrome [1,0,1,0] the parallel
    # schedule keeps every qubit's posterior identical (the ring's symmetries fix the syndrome
    # and act transitively on the qubits), so no flooding variant can converge.
    with open(os.path.join(GOLD, "paper_values.json")) as f:
        g = json.load(f)["trapping_set"]
    code = qecgen.trapping_ring()
    s = np.array(g["syndrome"], np.uint8)
    p = g["prior_probability"]
    pi = O.prior_llr(qecgen.depolarizing_probs(4, 3 * p))
    for variant, alpha in (("bp", 1.0), ("ewainit", 0.5), ("momentum", 0.5), ("adagrad", 5.0)):
        r = O.decode(code.hx, code.hz, O.Params(variant=variant, alpha=alpha, max_iter=g["max_iter"]),
                     pi, s[None], want_trace=True)
        assert r["conv"][0] == 0 and r["iters"][0] == g["max_iter"]
        qt = r["q_trace"][0]
        assert np.allclose(qt, qt[:, :1, :], rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# Exhaustive small-code decoding
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("make", [lambda: qecgen.planar(3), lambda: qecgen.toric(3),
                                  lambda: qecgen.xzzx(3)])
def test_all_weight_one_errors_are_corrected(make):
    # Distance 3: every weight-1 error has a unique minimum-weight explanation; each variant
    # returns exactly that error.
    code = make()
    errs = np.array([np.eye(code.n, dtype=np.uint8)[v] * P for v in range(code.n) for P in (1, 2, 3)])
    syn = syndrome_np(code.hx, code.hz, errs)
    pi = O.prior_llr(qecgen.depolarizing_probs(code.n, 0.05))
    for variant, alpha in (("bp", 1.0), ("ewainit", 0.5), ("momentum", 0.5), ("adagrad", 5.0)):
        r = O.decode(code.hx, code.hz, O.Params(variant=variant, alpha=alpha, max_iter=50), pi, syn)
        assert r["conv"].all()
        assert np.array_equal(r["est"], errs)
        _, counts = O.bookkeep(code.hx, code.hz, code.lx, code.lz, errs, r["est"])
        assert counts.tolist() == [len(errs), 0, 0]


def test_bookkeeping_classes():
    code = qecgen.planar(3)
    n = code.n
    stab = code.labels()[0]
    logical = (code.lx[0] | (code.lz[0] << 1)).astype(np.uint8)
    e = np.zeros(n, np.uint8)
    e[4] = 1
    errs = np.stack([e, e, e, e])
    ests = np.stack([e, e ^ stab, e ^ logical, np.zeros(n, np.uint8)])
    fail, counts = O.bookkeep(code.hx, code.hz, code.lx, code.lz, errs, ests)
    assert fail.tolist() == [0, 0, 2, 1]
    assert counts.tolist() == [2, 1, 1]


def _d3_exact(variant, alpha, p, max_iter=50):
    from tests.golden.make_d3_exact import exact_ler
    return exact_ler(variant, alpha, p, max_iter)


@pytest.mark.parametrize("variant,alpha", [("bp", 1.0), ("ewainit", 0.5)])
def test_d3_exact_ler_brackets_sampled(variant, alpha):
    # Config: planar d=3, depolarizing p = 0.05, iter_max 50.  The exact logical error rate of
    # the decoder (every syndrome, every coset) must lie in the CI of the 10^4-shot estimate,
    # and the exact maximum-likelihood rate bounds it from below.
    with open(os.path.join(GOLD, "d3_exact_ler.json")) as f:
        gold = json.load(f)
    key = f"{variant}_a{alpha}"
    exact, ml = _d3_exact(variant, alpha, 0.05)
    assert abs(exact - gold[key]["exact_ler"]) < 1e-12
    assert abs(ml - gold["ml_ler"]) < 1e-12
    assert ml <= exact + 1e-15
    code = qecgen.planar(3)
    thr = qecgen.thresholds(0.05 / 3, 0.05 / 3, 0.05 / 3)
    err, syn = O.sample(code.hx, code.hz, 10000, thr, seed=qecgen.config_seed(1, 0, 0))
    pi = O.prior_llr(qecgen.depolarizing_probs(code.n, 0.05))
    r = O.decode(code.hx, code.hz, O.Params(variant=variant, alpha=alpha, max_iter=50), pi, syn)
    _, counts = O.bookkeep(code.hx, code.hz, code.lx, code.lz, err, r["est"])
    lo, hi = O.wilson_ci(int(counts[1] + counts[2]), 10000, z=3.29)
    assert lo <= exact <= hi
