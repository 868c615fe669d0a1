"""GPU: the serial schedule (Algorithm 1) on the LDS kernel (level by level) and
the SOA kernel against the oracle, and the two kernels against each other bit for
bit.

Bar: messages and posteriors after iteration 1 (stopping off) within the 1e-5
bar of the flooding kernels; after iterations 2 and 3, at least 99.9% within
1e-5 and all within 1e-4 (one serial iteration chains the updates of every
qubit, so its rounding compounds like a much deeper flooding decode; measured:
one entry in 70,000 at 1.3e-5 after two iterations); AdaGrad from the third
iteration by the flooding kernels' quantile; decisions of shots converged on both sides >= 99.9% equal, LER in the
oracle's interval; AEWA attempts compose with the serial schedule.
"""
import sys

import numpy as np
import pytest

import qecgen
from oracle import oracle as O
from tests import bars
from tests.oracle_inputs import matched

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2407_11523_amd as P  # noqa: E402

REL_TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


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


@pytest.mark.parametrize("variant,alpha", [("bp", 1.0), ("ewainit", 0.5), ("momentum", 0.6), ("adagrad", 5.0)])
@pytest.mark.parametrize("T", [1, 2, 3])
def test_serial_messages(variant, alpha, T):
    x = qecgen.xzzx(5)
    for name, hx, hz in (("planar5", qecgen.planar(5).hx, qecgen.planar(5).hz),
                         ("xzzx5-clifford",) + clifford_relabel(x, 3)):
        n = hx.shape[1]
        g = P.Graph(hx, hz)
        probs = np.random.default_rng(5).uniform(0.01, 0.04, size=(n, 3))
        _, syn = O.sample(hx, hz, 700, qecgen.thresholds(*probs[0]), seed=13)
        ro = O.decode(hx, hz, O.Params(variant=variant, alpha=alpha, max_iter=T, stop_on_syndrome=False,
                                       serial=True), O.prior_llr(probs), syn, want_q=True, want_msgs=True,
                      want_trace=variant == "adagrad")
        prm = P.Params(variant=variant, alpha=alpha, max_iter=T, stop_on_syndrome=False, serial=True)
        rg = P.decode(g, prm, P.prior_llr(probs), torch.as_tensor(syn, device="cuda"), trace=True)
        rs = P.decode(g, prm, P.prior_llr(probs), torch.as_tensor(syn, device="cuda"), trace=True, kernel="soa")
        torch.cuda.synchronize()
        for k in ("est", "conv", "iters", "mvc", "mcv", "q"):   # LDS levels == SOA sweep, bit for bit
            assert torch.equal(rg[k], rs[k]), (name, variant, T, k)
        for k in ("mvc", "mcv", "q"):
            err = np.abs(np_(rg[k]).astype(np.float64) - ro[k]) / np.maximum(np.abs(ro[k]), 1.0)
            say("serial msg", name, variant, T, k, float(err.max()), float((err <= REL_TOL).mean()))
            if variant == "adagrad" and T >= 2:
                # eq. boost: the FP32 sign of a gradient near 0 decides a step of size alpha
                assert (err <= REL_TOL).mean() >= bars.ADAGRAD_SHARE, (name, k)
                if k == "q":
                    win = bars.adagrad_window_entries(ro["q_trace"], ro["m_trace"], O.prior_llr(probs))
                    say("serial adagrad window", name, T, bars.adagrad_report(err, win))
            elif T >= 2:
                assert (err <= REL_TOL).mean() >= 0.999 and err.max() <= 1e-4, (name, k)
            else:
                assert err.max() <= REL_TOL, (name, k)


@pytest.mark.parametrize("make,p,variant,alpha", [(lambda: qecgen.planar(7), 0.08, "ewainit", 0.5),
                                                  (lambda: qecgen.toric(8), 0.10, "momentum", 0.6),
                                                  (lambda: qecgen.planar(9), 0.06, "aewa", 1.0)])
def test_serial_decisions_and_ler(make, p, variant, alpha):
    code = make()
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    shots = 3000
    thr = qecgen.thresholds(p / 3, p / 3, p / 3)
    err, syn = P.sample(g, shots, thr, seed=41)
    kw = dict(variant=variant, alpha=alpha, max_iter=100, serial=True)
    if variant == "aewa":
        kw.update(alpha_last=0.0, alpha_steps=6)
    r = P.decode(g, P.Params(**kw), P.prior_llr(qecgen.depolarizing_probs(code.n, p)), syn)
    rs = P.decode(g, P.Params(**kw), P.prior_llr(qecgen.depolarizing_probs(code.n, p)), syn, kernel="soa")
    _, cnt = P.bookkeep(g, err, r["est"])
    torch.cuda.synchronize()
    for k in ("est", "conv", "iters"):
        assert torch.equal(r[k], rs[k]), k
    e_o, s_o = matched(code, thr, 41, err, syn)
    ro = O.decode(code.hx, code.hz, O.Params(**{k: v for k, v in kw.items()}),
                  O.prior_llr(qecgen.depolarizing_probs(code.n, p)), s_o)
    _, co = O.bookkeep(code.hx, code.hz, code.lx, code.lz, e_o, ro["est"])
    both = np_(r["conv"]).astype(bool) & ro["conv"].astype(bool)
    agree = float((np_(r["est"]) == ro["est"])[both].mean())
    ler_g = int(cnt[1] + cnt[2]) / shots
    lo, hi = O.wilson_ci(int(co[1] + co[2]), shots, z=3.29)
    say("serial", code.name, variant, dict(agree=agree, ler_g=ler_g, ler_o=int(co[1] + co[2]) / shots, ci=(lo, hi),
                                           iters_g=float(np_(r["iters"]).mean()), iters_o=float(ro["iters"].mean())))
    assert agree >= 0.999
    assert lo <= ler_g <= hi


def test_serial_rejected_where_unsupported():
    code = qecgen.planar(5)
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    syn = torch.zeros(10, code.m, dtype=torch.uint8, device="cuda")
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, 0.05))
    prm = P.Params(variant="ewainit", alpha=0.5, serial=True)
    for call in (lambda: P.decode_plain(g, prm, pr, syn), lambda: P.decode_mixed([(g, prm, pr, syn, 0)])):
        with pytest.raises(P.BP4Error) as e:
            call()
        assert e.value.name == "EUNSUPPORTED"
    for kw in (dict(block_shots=2), dict(group_lanes=128), dict(group_lanes=3)):
        with pytest.raises(P.BP4Error) as e:
            P.decode(g, prm, pr, syn, **kw)
        assert e.value.name == "EINVAL"


@pytest.mark.parametrize("make", [lambda: qecgen.toric(6), lambda: qecgen.xzzx(5)])
def test_serial_group_sizes_bitwise(make):
    """Every serial group size (including 1 and 2 lanes per shot) and the SOA sweep
    give the same bits; ragged shot counts."""
    code = make()
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, 0.1))
    for variant, kw in (("ewainit", dict(alpha=0.5)), ("aewa", dict(alpha=1.0, alpha_last=0.2, alpha_steps=4,
                                                                   max_iter=10))):
        prm = P.Params(variant=variant, serial=True, **dict(dict(max_iter=40), **kw))
        for shots in (1, 257, 2000):
            _, syn = P.sample(g, shots, qecgen.thresholds(0.1 / 3, 0.1 / 3, 0.1 / 3), seed=shots)
            ref = P.decode(g, prm, pr, syn, kernel="soa")
            for G in (1, 2, 4, 16, 64):
                try:
                    r = P.decode(g, prm, pr, syn, group_lanes=G)
                except P.BP4Error:      # LDS exhausted at this size
                    continue
                torch.cuda.synchronize()
                for k in ("est", "conv", "iters"):
                    assert torch.equal(r[k], ref[k]), (variant, shots, G, k)
