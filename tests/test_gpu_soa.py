"""GPU: the structure-of-arrays kernels for large codes (messages in HBM).

It runs the same per-node arithmetic as the LDS kernel, so on codes both can
decode its outputs must be bit-identical to the LDS kernel's; it is also held
to the oracle bar directly (messages at iterations 1..5, decisions and logical
error rates) and, on the large planar d=31 and toric L=32 codes at the full
2^18-shot batch (decoded by the single-pass HBM kernel the benchmark times, and
bit-identical to the two-phase kernel), on a sample of shots that the oracle
decodes one by one.
"""
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
VARIANTS = [("bp", 1.0), ("ewainit", 0.5), ("momentum", 0.6), ("adagrad", 5.0)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def np_(t):
    return t.detach().cpu().numpy()


def check_msgs(r, variant, T):
    """Every message and posterior within 1e-5; AdaGrad (eq. boost, T >= 2): at least
    99.9% of the entries of each kind within 1e-5."""
    if variant == "adagrad" and T >= 2:
        for k in ("mvc", "mcv", "q"):
            assert r[k + "_frac_1e-5"] >= bars.ADAGRAD_SHARE, (k, r)
    else:
        for k in ("mvc", "mcv", "q"):
            assert r[k] <= REL_TOL, (k, r)


def clifford_relabel(code, seed):
    rng = np.random.default_rng(seed)
    lab = code.labels()
    new = np.zeros_like(lab)
    for v in range(code.n):
        p = rng.permutation([1, 2, 3])
        mp = np.array([0, p[0], p[1], p[2]], np.uint8)
        new[:, v] = mp[lab[:, v]]
    return (new & 1).astype(np.uint8), (new >> 1).astype(np.uint8)


def msg_parity(hx, hz, lx, lz, probs, shots, seed, variant, alpha, T):
    g = P.Graph(hx, hz, lx, lz)
    thr = qecgen.thresholds(*probs[0])
    _, syn = O.sample(hx, hz, shots, thr, seed=seed)
    prm_o = O.Params(variant=variant, alpha=alpha, max_iter=T, stop_on_syndrome=False)
    prm_g = P.Params(variant=variant, alpha=alpha, max_iter=T, stop_on_syndrome=False)
    pi = O.prior_llr(probs)
    ro = O.decode(hx, hz, prm_o, pi, syn, want_q=True, want_msgs=True, want_trace=variant == "adagrad")
    rg = P.decode(g, prm_g, P.prior_llr(probs), torch.as_tensor(syn, device="cuda"), trace=True, kernel="soa")
    torch.cuda.synchronize()
    out = {}
    for k in ("mvc", "mcv", "q"):
        err = bars.rel_err(np_(rg[k]), ro[k])
        out[k] = float(err.max())
        out[k + "_frac_1e-5"] = float((err <= REL_TOL).mean())
        if k == "q" and variant == "adagrad" and T >= 2:
            win = bars.adagrad_window_entries(ro["q_trace"], ro["m_trace"], pi)
            rep = bars.adagrad_report(err, win)
            out["q_window_frac"], out["q_outside_window"] = rep["window_frac"], rep["outside_max"]
            out["q_in_window_frac_1e-5"] = rep["inside_frac_1e5"]
    out["iters_equal"] = bool(np.array_equal(np_(rg["iters"]), ro["iters"]))
    return out


@pytest.mark.parametrize("variant,alpha", VARIANTS)
@pytest.mark.parametrize("T", [1, 2, 3, 5])
def test_soa_messages_planar_d3(variant, alpha, T):
    code = qecgen.planar(3)
    probs = qecgen.depolarizing_probs(code.n, 0.05)
    # 2000 shots: the last workgroup of lanes is ragged
    r = msg_parity(code.hx, code.hz, code.lx, code.lz, probs, 2000, 11, variant, alpha, T)
    say("soa msg planar3", variant, T, r)
    check_msgs(r, variant, T)
    assert r["iters_equal"]


@pytest.mark.parametrize("variant,alpha", VARIANTS)
def test_soa_messages_y_labels(variant, alpha):
    # Y labels and non-uniform priors: random local Cliffords on the XZZX code
    x = qecgen.xzzx(5)
    hx, hz = clifford_relabel(x, 3)
    rng = np.random.default_rng(5)
    probs = rng.uniform(0.01, 0.04, size=(x.n, 3))
    r = msg_parity(hx, hz, x.lx, x.lz, probs, 1024, 13, variant, alpha, 5)
    say("soa msg xzzx5-clifford", variant, r)
    check_msgs(r, variant, 5)


def _run(g, prm, pr, syn, kernel, trace=False):
    r = P.decode(g, prm, pr, syn, kernel=kernel, trace=trace)
    torch.cuda.synchronize()
    return r


@pytest.mark.parametrize("make,variant,alpha", [(lambda: qecgen.planar(9), "ewainit", 0.5),
                                                (lambda: qecgen.toric(10), "bp", 1.0),
                                                (lambda: qecgen.xzzx(9), "momentum", 0.6),
                                                (lambda: qecgen.planar(13), "adagrad", 5.0)])
def test_soa_equals_lds_bitwise(make, variant, alpha):
    code = make()
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    p = 0.08
    _, syn = P.sample(g, 20000, qecgen.thresholds(p / 3, p / 3, p / 3), seed=51)
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p))
    prm = P.Params(variant=variant, alpha=alpha, max_iter=60)
    a = _run(g, prm, pr, syn, "lds")
    b = _run(g, prm, pr, syn, "soa")
    say("soa==lds", code.name, variant, float(a["iters"].float().mean()))
    for k in ("est", "conv", "iters"):
        assert torch.equal(a[k], b[k]), k
    # every message and posterior after five iterations without stopping
    prm5 = P.Params(variant=variant, alpha=alpha, max_iter=5, stop_on_syndrome=False)
    a = _run(g, prm5, pr, syn[:3000], "lds", trace=True)
    b = _run(g, prm5, pr, syn[:3000], "soa", trace=True)
    for k in ("q", "mvc", "mcv", "est"):
        assert torch.equal(a[k], b[k]), k


def test_soa_lane_reuse_and_ragged():
    # more shots than resident lanes: lanes take new shots from the queue in place
    code = qecgen.planar(3)
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    p = 0.1
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p))
    prm = P.Params(variant="ewainit", alpha=0.5, max_iter=50)
    for shots in (1, 63, 300, (1 << 18) + 4097):
        _, syn = P.sample(g, shots, qecgen.thresholds(p / 3, p / 3, p / 3), seed=shots)
        a = _run(g, prm, pr, syn, "lds")
        b = _run(g, prm, pr, syn, "soa")
        say("soa ragged", shots)
        for k in ("est", "conv", "iters"):
            assert torch.equal(a[k], b[k]), (shots, k)
    # zero shots: nothing launched, nothing written
    z = torch.empty(0, code.m, dtype=torch.uint8, device="cuda")
    r = _run(g, prm, pr, z, "soa")
    assert r["est"].shape == (0, code.n)


def test_soa_block_length_and_lanes_do_not_change_results():
    # iteration blocks of any length, lanes fewer than shots (several chunks, each
    # packed between blocks): bit-identical to the LDS kernel
    code = qecgen.xzzx(9)
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    p = 0.12
    _, syn = P.sample(g, 5000, qecgen.thresholds(p / 3, p / 3, p / 3), seed=77)
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p))
    prm = P.Params(variant="momentum", alpha=0.6, gamma=0.3, max_iter=45)
    ref = _run(g, prm, pr, syn, "lds")
    for block, lanes in ((1, 0), (7, 0), (16, 1024), (45, 256), (200, 2048)):
        r = P.decode(g, prm, pr, syn, kernel="soa", soa_iter_block=block, soa_lanes=lanes)
        torch.cuda.synchronize()
        say("soa block", block, "lanes", lanes)
        for k in ("est", "conv", "iters"):
            assert torch.equal(ref[k], r[k]), (block, lanes, k)


def test_soa_moved_columns_keep_every_message():
    """Blocks of 3 iterations without stopping: the last iteration of each block
    writes the shots' new columns; messages and posteriors after 10 iterations
    equal the LDS kernel's bit for bit (AdaGrad keeps a second state array)."""
    code = qecgen.planar(7)
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    p = 0.1
    _, syn = P.sample(g, 3000, qecgen.thresholds(p / 3, p / 3, p / 3), seed=19)
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p))
    for variant, alpha in (("ewainit", 0.5), ("adagrad", 5.0)):
        prm = P.Params(variant=variant, alpha=alpha, max_iter=10, stop_on_syndrome=False)
        a = _run(g, prm, pr, syn, "lds", trace=True)
        b = P.decode(g, prm, pr, syn, kernel="soa", trace=True, soa_iter_block=3, soa_lanes=1024)
        torch.cuda.synchronize()
        say("soa moved columns", variant)
        for k in ("q", "mvc", "mcv", "est", "conv", "iters"):
            assert torch.equal(a[k], b[k]), (variant, k)


def test_soa_workspace_checked():
    code = qecgen.planar(5)
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    prm = P.Params(variant="momentum", alpha=0.6, max_iter=5)
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, 0.05))
    syn = torch.zeros(1000, code.m, dtype=torch.uint8, device="cuda")
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.BP4Error):
        P.decode(g, prm, pr, syn, kernel="soa", ws=small)


@pytest.mark.parametrize("make", [lambda: qecgen.planar(31), lambda: qecgen.toric(32)])
@pytest.mark.parametrize("variant,alpha", VARIANTS)
def test_soa_messages_large_codes(make, variant, alpha):
    code = make()
    probs = qecgen.depolarizing_probs(code.n, 0.10)
    for T in (1, 3, 5):
        r = msg_parity(code.hx, code.hz, code.lx, code.lz, probs, 300, 17, variant, alpha, T)
        say("soa msg", code.name, variant, T, r)
        check_msgs(r, variant, T)


@pytest.mark.parametrize("make", [lambda: qecgen.planar(31), lambda: qecgen.toric(32)])
def test_large_codes_full_batch_sampled(make):
    """The full 2^18-shot batch at p = 0.10, EWAInit with the chosen discount, max 200
    iterations, in the launch the benchmark times (the single-pass HBM kernel, which
    must also equal the two-phase SOA kernel bit for bit on the whole batch); 192 shots
    spread over the batch decoded by the oracle.

    Near threshold most shots run for 100+ iterations and the map from priors to
    decisions is sensitive: the oracle itself, given priors perturbed by a relative
    1e-7 (FP32 rounding), does not reproduce all of its decisions.  The GPU is held
    to that same agreement minus a 3-sigma sampling margin (or 99.9% where that is
    lower), to exact agreement on shots that converge within 20 iterations, and its
    logical error rate over the whole batch to the oracle's interval on the sample."""
    code = make()
    shots = configs.CONFIG5["shots"]
    p, max_iter = configs.CONFIG5["p"], configs.CONFIG5["max_iter"]
    alpha = configs.alpha(5, "ewainit")
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([[0, 1, shots - 1], rng.choice(shots, 189, replace=False)]))
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    thr = qecgen.thresholds(p / 3, p / 3, p / 3)
    seed = qecgen.config_seed(5, 0 if code.name.startswith("planar") else 1, 0)
    err, syn = P.sample(g, shots, thr, seed=seed)
    prm = P.Params(variant="ewainit", alpha=alpha, max_iter=max_iter)
    say("large", code.name, shots, "alpha", alpha, "workspace", g.workspace_bytes(prm, shots))
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p))
    rg = P.decode(g, prm, pr, syn, kernel="gather")
    fail_g, cnt_g = P.bookkeep(g, err, rg["est"])
    torch.cuda.synchronize()
    rs = P.decode(g, prm, pr, syn, kernel="soa")
    torch.cuda.synchronize()
    for k in ("est", "conv", "iters"):
        assert torch.equal(rg[k], rs[k]), k
    del rs
    sel = torch.as_tensor(idx, device=syn.device)
    e, s = matched(code, thr, seed, err, syn, idx=idx)
    est_g, conv_g, it_g = np_(rg["est"][sel]), np_(rg["conv"][sel]), np_(rg["iters"][sel])
    pi = O.prior_llr(qecgen.depolarizing_probs(code.n, p))
    op = O.Params(variant="ewainit", alpha=alpha, max_iter=max_iter)
    bar = bars.decision_bar(code, op, pi, s, est_g)
    ro = bar.pop("ro")
    bar.pop("rp")
    early = bars.early_exact(est_g, conv_g, it_g, ro)
    assert np.array_equal(it_g[early], ro["iters"][early])
    _, cnt_o = O.bookkeep(code.hx, code.hz, code.lx, code.lz, e, ro["est"])
    ler_g = int(cnt_g[1] + cnt_g[2]) / shots
    ci_o = O.wilson_ci(int(cnt_o[1] + cnt_o[2]), len(idx), z=3.29)
    say("large", code.name, dict(bar, early=int(early.sum()), conv_g=float(np_(rg["conv"]).mean()),
                                 iters_g=float(np_(rg["iters"]).mean()), ler_g=ler_g, ci_o=ci_o))
    assert bar["ok"], bar
    assert ci_o[0] <= ler_g <= ci_o[1]
