"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bar: bit-exact for sampling, syndromes and bookkeeping; messages within
|m32 - m64| <= 1e-5 max(|m64|, 1) at iterations 1..5 with stopping off; at
least 99.9% identical hard decisions (or, where the FP64 oracle disagrees
with itself under a 1e-7 prior perturbation by more, that measured agreement
minus a sampling margin); logical error rates inside each other's Wilson 95%
interval.  AdaGrad (eq. boost): at least 99.9% of the message and posterior
entries within 1e-5, the share whose FP64 gradient entered the kernels'
deadband window reported.
"""
import math
import sys

import numpy as np
import pytest

import qecgen
from oracle import oracle as O
from qecgen import configs
from tests import bars
from tests.oracle_inputs import matched

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2407_11523_amd as P  # noqa: E402

REL_TOL = bars.REL_TOL


def check_msgs(r, variant, T):
    """Every message and posterior within 1e-5; AdaGrad (eq. boost, T >= 2): at least
    99.9% of the entries of each kind within 1e-5 (the FP32 sign of a gradient near 0
    decides a step of size alpha), with the share in the deadband window reported."""
    if variant == "adagrad" and T >= 2:
        for k in ("mvc", "mcv", "q"):
            assert r[k + "_frac_1e-5"] >= bars.ADAGRAD_SHARE, (k, r)
    else:
        for k in ("mvc", "mcv", "q"):
            assert r[k] <= REL_TOL, (k, r)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_graph(code):
    return P.Graph(code.hx, code.hz, code.lx, code.lz)


def np_(t):
    return t.detach().cpu().numpy()


def clifford_relabel(code, seed):
    rng = np.random.default_rng(seed)
    lab = code.labels()
    new = np.zeros_like(lab)
    for v in range(code.n):
        p = rng.permutation([1, 2, 3])
        mp = np.array([0, p[0], p[1], p[2]], np.uint8)
        new[:, v] = mp[lab[:, v]]
    return (new & 1).astype(np.uint8), (new >> 1).astype(np.uint8)


# ---------------------------------------------------------------------------
# Integer work: bit-exact
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("make,shots,shot0", [(lambda: qecgen.planar(3), 1000, 0),
                                             (lambda: qecgen.toric(8), 4096, 12345),
                                             (lambda: qecgen.xzzx(5), 777, 3),
                                             (lambda: qecgen.planar(31), 64, 99)])
def test_sample_bit_exact(make, shots, shot0):
    code = make()
    say("sample", code.name, shots, shot0)
    g = gpu_graph(code)
    thr = qecgen.thresholds(0.03, 0.02, 0.05)
    err, syn = P.sample(g, shots, thr, seed=2024, stream_id=7, shot0=shot0)
    torch.cuda.synchronize()
    e0, s0 = O.sample(code.hx, code.hz, shots, thr, seed=2024, stream=7, shot0=shot0)
    assert np.array_equal(np_(err), e0)
    assert np.array_equal(np_(syn), s0)


def test_sample_zero_shots():
    code = qecgen.toric(4)
    g = gpu_graph(code)
    err, syn = P.sample(g, 0, qecgen.thresholds(0.01, 0.01, 0.01), seed=1)
    torch.cuda.synchronize()
    assert err.shape == (0, code.n) and syn.shape == (0, code.m)


@pytest.mark.parametrize("make", [lambda: qecgen.planar(5), lambda: qecgen.toric(6), lambda: qecgen.xzzx(9),
                                  lambda: qecgen.planar(31)])
def test_bookkeep_bit_exact(make):
    code = make()
    say("bookkeep", code.name)
    g = gpu_graph(code)
    rng = np.random.default_rng(4)
    shots = 3000 if code.n < 1000 else 200
    err = rng.integers(0, 4, size=(shots, code.n)).astype(np.uint8) * (rng.random((shots, code.n)) < 0.05)
    est = err.copy()
    # a third unchanged, a third multiplied by a stabilizer or logical, a third random
    lab = code.labels()
    logical = (code.lx | (code.lz << 1)).astype(np.uint8)
    for i in range(shots):
        k = i % 3
        if k == 1:
            est[i] ^= lab[rng.integers(code.m)]
            if rng.random() < 0.5:
                est[i] ^= logical[rng.integers(len(logical))]
        elif k == 2:
            est[i] = rng.integers(0, 4, size=code.n) * (rng.random(code.n) < 0.03)
    fail_o, cnt_o = O.bookkeep(code.hx, code.hz, code.lx, code.lz, err, est)
    fail_g, cnt_g = P.bookkeep(g, torch.as_tensor(err, device="cuda"), torch.as_tensor(est, device="cuda"))
    torch.cuda.synchronize()
    assert np.array_equal(np_(fail_g), fail_o)
    assert np_(cnt_g).tolist() == cnt_o.tolist()
    assert cnt_o[2] > 0 and cnt_o[1] > 0 and cnt_o[0] > 0


def test_sample_and_bookkeep_on_unaligned_views():
    """Rows that start off a 4-byte boundary (slices of a caller's buffers): the
    staged row copies of the syndrome and bookkeeping kernels take their byte path
    at both ends and for an unaligned second operand; results stay bit-exact."""
    code = qecgen.planar(5)   # n = 41, m = 40
    say("unaligned views", code.name)
    g = gpu_graph(code)
    shots = 1000
    thr = qecgen.thresholds(0.03, 0.02, 0.05)
    ebuf = torch.zeros(shots + 1, code.n, dtype=torch.uint8, device="cuda")
    sbuf = torch.zeros(shots * code.m + 3, dtype=torch.uint8, device="cuda")
    err = ebuf[1:]                                   # starts 41 bytes in
    syn = sbuf[3:].view(shots, code.m)               # starts 3 bytes in
    P.sample(g, shots, thr, seed=77, stream_id=1, err=err, synd=syn)
    torch.cuda.synchronize()
    e0, s0 = O.sample(code.hx, code.hz, shots, thr, seed=77, stream=1, shot0=0)
    assert np.array_equal(np_(err), e0) and np.array_equal(np_(syn), s0)
    rng = np.random.default_rng(5)
    est = e0 ^ (rng.integers(0, 4, size=e0.shape) * (rng.random(e0.shape) < 0.02)).astype(np.uint8)
    est_buf = torch.zeros(shots + 2, code.n, dtype=torch.uint8, device="cuda")
    est_buf[2:] = torch.as_tensor(est, device="cuda")
    fail_g, cnt_g = P.bookkeep(g, err, est_buf[2:])  # 82 bytes in: 2-byte aligned
    torch.cuda.synchronize()
    fail_o, cnt_o = O.bookkeep(code.hx, code.hz, code.lx, code.lz, e0, est)
    assert np.array_equal(np_(fail_g), fail_o)
    assert np_(cnt_g).tolist() == cnt_o.tolist()
    assert cnt_o[1] > 0 and cnt_o[0] > 0


# ---------------------------------------------------------------------------
# Messages at iterations 1..5 (stopping off) against FP64
# ---------------------------------------------------------------------------

VARIANTS = [("bp", 1.0), ("ewainit", 0.5), ("momentum", 0.6), ("adagrad", 5.0)]


def _msg_parity(code_hx, code_hz, lx, lz, probs, shots, seed, variant, alpha, T, group_lanes=0,
                gamma=0.0):
    g = P.Graph(code_hx, code_hz, lx, lz)
    thr = qecgen.thresholds(*probs[0])
    _, syn = O.sample(code_hx, code_hz, shots, thr, seed=seed)
    pi64 = O.prior_llr(probs)
    pi32 = P.prior_llr(probs)
    prm_o = O.Params(variant=variant, alpha=alpha, gamma=gamma, max_iter=T, stop_on_syndrome=False)
    prm_g = P.Params(variant=variant, alpha=alpha, gamma=gamma, max_iter=T, stop_on_syndrome=False)
    ro = O.decode(code_hx, code_hz, prm_o, pi64, syn, want_q=True, want_msgs=True, want_trace=variant == "adagrad")
    rg = P.decode(g, prm_g, pi32, torch.as_tensor(syn, device="cuda"), trace=True, group_lanes=group_lanes)
    torch.cuda.synchronize()
    out = {}
    for k64, k32 in (("mvc", "mvc"), ("mcv", "mcv"), ("q", "q")):
        a = ro[k64]
        b = np_(rg[k32]).astype(np.float64)
        err = np.abs(b - a) / np.maximum(np.abs(a), 1.0)
        out[k64] = float(err.max())
        out[k64 + "_frac_1e-5"] = float((err <= REL_TOL).mean())
        if k64 == "q" and variant == "adagrad" and T >= 2:
            win = bars.adagrad_window_entries(ro["q_trace"], ro["m_trace"], pi64)
            out["q_window_frac"] = float(win.mean())
            out["q_outside_window"] = float(err[~win].max()) if (~win).any() else 0.0
            out["q_in_window_frac_1e-5"] = float((err[win] <= REL_TOL).mean()) if win.any() else 1.0
    out["iters_equal"] = bool(np.array_equal(np_(rg["iters"]), ro["iters"]))
    out["est_agree"] = float((np_(rg["est"]) == ro["est"]).mean())
    return out


@pytest.mark.parametrize("variant,alpha", VARIANTS)
@pytest.mark.parametrize("T", [1, 2, 3, 5])
def test_messages_planar_d3(variant, alpha, T):
    code = qecgen.planar(3)
    probs = qecgen.depolarizing_probs(code.n, 0.05)
    r = _msg_parity(code.hx, code.hz, code.lx, code.lz, probs, 2000, 11, variant, alpha, T)
    say("msg planar3", variant, T, r)
    check_msgs(r, variant, T)
    assert r["iters_equal"]


@pytest.mark.parametrize("variant,alpha", VARIANTS)
def test_messages_toric_l8_and_relabelled(variant, alpha):
    code = qecgen.toric(8)
    probs = qecgen.depolarizing_probs(code.n, 0.08)
    r = _msg_parity(code.hx, code.hz, code.lx, code.lz, probs, 1024, 12, variant, alpha, 5)
    say("msg toric8", variant, r)
    check_msgs(r, variant, 5)
    # Y labels and non-uniform priors: random local Cliffords on the XZZX code
    x = qecgen.xzzx(5)
    hx, hz = clifford_relabel(x, 3)
    rng = np.random.default_rng(5)
    probs = rng.uniform(0.01, 0.04, size=(x.n, 3))
    r = _msg_parity(hx, hz, x.lx, x.lz, probs, 1024, 13, variant, alpha, 5)
    say("msg xzzx5-clifford", variant, r)
    check_msgs(r, variant, 5)


@pytest.mark.parametrize("gamma,alpha", [(0.3, 0.6), (0.7, 0.5)])
@pytest.mark.parametrize("T", [1, 2, 3, 4, 5])
def test_momentum_with_decay_against_oracle(gamma, alpha, T):
    # eqs. mombp1-3 with gamma != 0: the momentum buffer carries earlier gradients
    code = qecgen.planar(3)
    probs = qecgen.depolarizing_probs(code.n, 0.05)
    r = _msg_parity(code.hx, code.hz, code.lx, code.lz, probs, 2000, 15, "momentum", alpha, T, gamma=gamma)
    say("msg planar3 momentum", gamma, T, r)
    check_msgs(r, "momentum", T)
    assert r["iters_equal"]
    code = qecgen.toric(8)
    r = _msg_parity(code.hx, code.hz, code.lx, code.lz, qecgen.depolarizing_probs(code.n, 0.08), 1024, 16,
                    "momentum", alpha, T, gamma=gamma)
    say("msg toric8 momentum", gamma, T, r)
    check_msgs(r, "momentum", T)
    x = qecgen.xzzx(5)
    hx, hz = clifford_relabel(x, 4)
    probs = np.random.default_rng(6).uniform(0.01, 0.04, size=(x.n, 3))
    r = _msg_parity(hx, hz, x.lx, x.lz, probs, 1024, 17, "momentum", alpha, T, gamma=gamma)
    say("msg xzzx5-clifford momentum", gamma, T, r)
    check_msgs(r, "momentum", T)


@pytest.mark.parametrize("G", [4, 8, 16, 32, 64, 128, 256])
def test_every_group_size(G):
    # one code per lane-group size, including ragged tails (m, n not multiples of G)
    code = qecgen.planar(7) if G >= 16 else qecgen.planar(3)
    probs = qecgen.depolarizing_probs(code.n, 0.06)
    r = _msg_parity(code.hx, code.hz, code.lx, code.lz, probs, 777, 14, "ewainit", 0.7, 4, group_lanes=G)
    say("group", G, code.name, r)
    assert r["mvc"] <= REL_TOL and r["mcv"] <= REL_TOL and r["q"] <= REL_TOL


# ---------------------------------------------------------------------------
# Decisions and logical error rates with early stopping
# ---------------------------------------------------------------------------

def _ler_parity(code, p, shots, variant, alpha, max_iter, seed, group_lanes=0, oracle_shots=None):
    g = gpu_graph(code)
    thr = qecgen.thresholds(p / 3, p / 3, p / 3)
    err, syn = P.sample(g, shots, thr, seed=seed)
    prm = P.Params(variant=variant, alpha=alpha, max_iter=max_iter)
    rg = P.decode(g, prm, P.prior_llr(qecgen.depolarizing_probs(code.n, p)), syn, group_lanes=group_lanes)
    fail_g, cnt_g = P.bookkeep(g, err, rg["est"])
    torch.cuda.synchronize()
    k = oracle_shots or shots
    e_o, s_o = matched(code, thr, seed, err[:k], syn[:k])
    pi = O.prior_llr(qecgen.depolarizing_probs(code.n, p))
    op = O.Params(variant=variant, alpha=alpha, max_iter=max_iter)
    est_g, conv_g, it_g = np_(rg["est"][:k]), np_(rg["conv"][:k]), np_(rg["iters"][:k])
    bar = bars.decision_bar(code, op, pi, s_o, est_g)
    ro = bar.pop("ro")
    bar.pop("rp")
    early = bars.early_exact(est_g, conv_g, it_g, ro)
    f_o, cnt_o = O.bookkeep(code.hx, code.hz, code.lx, code.lz, e_o, ro["est"])
    ler_g = int(cnt_g[1] + cnt_g[2]) / shots
    ler_o = int(cnt_o[1] + cnt_o[2]) / k
    ci_g = O.wilson_ci(int(cnt_g[1] + cnt_g[2]), shots)
    ci_o = O.wilson_ci(int(cnt_o[1] + cnt_o[2]), k)
    return dict(bar=bar, early=int(early.sum()), ler_g=ler_g, ler_o=ler_o, ci_g=ci_g, ci_o=ci_o,
                iters_g=float(np_(rg["iters"]).mean()), iters_o=float(ro["iters"].mean()),
                same_iters=float((it_g == ro["iters"]).mean()),
                conv_g=float(np_(rg["conv"]).mean()), conv_o=float(ro["conv"].mean()))


@pytest.mark.parametrize("variant", ["bp", "ewainit"])
def test_config1_planar_d3(variant):
    # planar d=3, depolarizing p=0.05, 10^4 shots, iter_max 50
    c1 = configs.CONFIG1
    r = _ler_parity(qecgen.make(c1["family"], c1["size"]), c1["p"], c1["shots"], variant,
                    configs.alpha(1, variant), c1["max_iter"], qecgen.config_seed(1, 0, 0))
    say("config1", variant, r)
    assert r["bar"]["ok"] and r["bar"]["gpu"] >= 0.999, r
    assert r["ci_o"][0] <= r["ler_g"] <= r["ci_o"][1]
    assert r["ci_g"][0] <= r["ler_o"] <= r["ci_g"][1]


def test_edge_cases():
    code = qecgen.toric(6)
    g = gpu_graph(code)
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, 0.05))
    # zero syndrome converges at t = 1 to the identity
    syn = torch.zeros((300, code.m), dtype=torch.uint8, device="cuda")
    r = P.decode(g, P.Params(variant="ewainit", alpha=0.5, max_iter=10), pr, syn)
    torch.cuda.synchronize()
    assert np_(r["conv"]).all() and (np_(r["iters"]) == 1).all() and not np_(r["est"]).any()
    # zero shots
    r = P.decode(g, P.Params(), pr, torch.zeros((0, code.m), dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    assert r["est"].shape == (0, code.n)
    # max_iter = 1 and a single shot
    thr = qecgen.thresholds(0.03, 0.03, 0.03)
    e, s = P.sample(g, 1, thr, seed=3)
    r = P.decode(g, P.Params(max_iter=1), pr, s)
    torch.cuda.synchronize()
    _, so = O.sample(code.hx, code.hz, 1, thr, seed=3)
    ro = O.decode(code.hx, code.hz, O.Params(max_iter=1), O.prior_llr(qecgen.depolarizing_probs(code.n, 0.05)), so)
    assert np_(r["iters"]).tolist() == [1] and np.array_equal(np_(r["est"]), ro["est"])
    # determinism: two runs are bit-identical
    e, s = P.sample(g, 5000, thr, seed=4)
    a = P.decode(g, P.Params(variant="ewainit", alpha=0.5), pr, s)
    b = P.decode(g, P.Params(variant="ewainit", alpha=0.5), pr, s)
    torch.cuda.synchronize()
    for k in ("est", "conv", "iters"):
        assert torch.equal(a[k], b[k])


def toric_translation(L, a, b):
    """Qubit and check permutations of the toric code under a lattice translation."""
    n = 2 * L * L
    qp = np.zeros(n, int)
    cp = np.zeros(n, int)
    for i in range(L):
        for j in range(L):
            t = ((i + a) % L) * L + (j + b) % L
            qp[i * L + j] = t
            qp[L * L + i * L + j] = L * L + t
            cp[i * L + j] = t
            cp[L * L + i * L + j] = L * L + t
    return qp, cp


@pytest.mark.parametrize("variant,alpha", VARIANTS)
def test_toric_translation_equivariance_bitwise(variant, alpha):
    # Translating the syndrome on the torus translates the decoder's output exactly: the
    # kernel's sums are formed in value order or per label, so a graph automorphism that
    # fixes the labels maps every intermediate value to a bitwise-equal one.
    L = 8
    code = qecgen.toric(L)
    qp, cp = toric_translation(L, 3, 5)
    hx2 = np.zeros_like(code.hx)
    hx2[cp[:, None], qp[None, :]] = code.hx
    assert np.array_equal(hx2, code.hx)
    g = gpu_graph(code)
    thr = qecgen.thresholds(0.08 / 3, 0.08 / 3, 0.08 / 3)
    _, syn = P.sample(g, 4096, thr, seed=31)
    syn2 = torch.empty_like(syn)
    syn2[:, torch.as_tensor(cp, device="cuda")] = syn
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, 0.08))
    prm = P.Params(variant=variant, alpha=alpha, max_iter=100)
    a = P.decode(g, prm, pr, syn)
    b = P.decode(g, prm, pr, syn2)
    torch.cuda.synchronize()
    assert torch.equal(a["iters"], b["iters"]) and torch.equal(a["conv"], b["conv"])
    assert torch.equal(b["est"][:, torch.as_tensor(qp, device="cuda")], a["est"])


def test_trapping_ring_never_converges_gpu():
    # Section IV-A, Table I: the ring's symmetries keep every qubit's posterior equal under
    # the flooding schedule; the GPU keeps them bitwise equal, so no variant converges.
    code = qecgen.trapping_ring()
    g = gpu_graph(code)
    pr = P.prior_llr(qecgen.depolarizing_probs(4, 0.03))
    syn = torch.as_tensor(np.array([[1, 0, 1, 0]], np.uint8), device="cuda")
    for variant, alpha in VARIANTS:
        r = P.decode(g, P.Params(variant=variant, alpha=alpha, max_iter=50), pr, syn, trace=True)
        torch.cuda.synchronize()
        assert np_(r["conv"]).tolist() == [0] and np_(r["iters"]).tolist() == [50]
        q = np_(r["q"])[0]
        assert (q == q[:1]).all(), variant
