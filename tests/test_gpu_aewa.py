"""GPU: AEWA-BP (EWAInit-BP restarted over a list of discounts until the syndrome
is met) in the persistent LDS kernel and the large-code SOA kernel.

Bar: against the FP64 oracle, decisions and attempt-summed iteration counts of
shots that converge on both sides agree (>= 99.9% / >= 99%), LER inside the
oracle's interval; the two kernels and the mixed launch agree bit for bit.
"""
import sys

import numpy as np
import pytest

import qecgen
from oracle import oracle as O
from tests.oracle_inputs import matched

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2407_11523_amd as P  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def np_(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("make,p,shots", [(lambda: qecgen.planar(7), 0.09, 4000),
                                          (lambda: qecgen.planar(11), 0.06, 2000),
                                          (lambda: qecgen.toric(8), 0.10, 600)])
def test_aewa_vs_oracle(make, p, shots):
    code = make()
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    thr = qecgen.thresholds(p / 3, p / 3, p / 3)
    err, syn = P.sample(g, shots, thr, seed=17)
    prm = P.Params(variant="aewa", alpha=1.0, alpha_last=0.0, alpha_steps=11, max_iter=100)
    r = P.decode(g, prm, P.prior_llr(qecgen.depolarizing_probs(code.n, p)), syn)
    _, cnt = P.bookkeep(g, err, r["est"])
    torch.cuda.synchronize()
    e_o, s_o = matched(code, thr, 17, err, syn)
    ro = O.decode(code.hx, code.hz, O.Params(variant="aewa", alpha=1.0, alpha_last=0.0, alpha_steps=11,
                                             max_iter=100),
                  O.prior_llr(qecgen.depolarizing_probs(code.n, p)), s_o)
    _, co = O.bookkeep(code.hx, code.hz, code.lx, code.lz, e_o, ro["est"])
    both = np_(r["conv"]).astype(bool) & ro["conv"].astype(bool)
    agree = float((np_(r["est"]) == ro["est"])[both].mean())
    it_agree = float((np_(r["iters"]) == ro["iters"])[both].mean())
    ler_g, ler_o = int(cnt[1] + cnt[2]) / shots, int(co[1] + co[2]) / shots
    lo, hi = O.wilson_ci(int(co[1] + co[2]), shots, z=3.29)
    restarted = float((np_(r["iters"]) > 100).mean())
    say("aewa", code.name, dict(agree=agree, it_agree=it_agree, ler_g=ler_g, ler_o=ler_o, ci=(lo, hi),
                                conv_g=float(np_(r["conv"]).mean()), restarted=restarted))
    assert restarted > 0
    assert agree >= 0.999 and it_agree >= 0.99
    assert lo <= ler_g <= hi


def test_aewa_lds_soa_and_mixed_bitwise():
    code = qecgen.planar(9)
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    p = 0.1
    err, syn = P.sample(g, 3000, qecgen.thresholds(p / 3, p / 3, p / 3), seed=23)
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p))
    prm = P.Params(variant="aewa", alpha=1.0, alpha_last=0.2, alpha_steps=5, max_iter=40)
    a = P.decode(g, prm, pr, syn, kernel="lds")
    b = P.decode(g, prm, pr, syn, kernel="soa", soa_lanes=1024, soa_iter_block=7)
    c2 = qecgen.toric(6)
    g2 = P.Graph(c2.hx, c2.hz, c2.lx, c2.lz)
    _, syn2 = P.sample(g2, 2000, qecgen.thresholds(p / 3, p / 3, p / 3), seed=24)
    pr2 = P.prior_llr(qecgen.depolarizing_probs(c2.n, p))
    prm2 = P.Params(variant="ewainit", alpha=0.5, max_iter=40)
    mixed = P.decode_mixed([(g, prm, pr, syn, 0), (g2, prm2, pr2, syn2, 0)])
    single2 = P.decode(g2, prm2, pr2, syn2)
    torch.cuda.synchronize()
    say("aewa bitwise", float(a["iters"].float().mean()), int((a["iters"] > 40).sum()))
    assert int((a["iters"] > 40).sum()) > 0
    for k in ("est", "conv", "iters"):
        assert torch.equal(a[k], b[k]), k
        assert torch.equal(a[k], mixed[0][k]), k
        assert torch.equal(single2[k], mixed[1][k]), k
