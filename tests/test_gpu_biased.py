"""GPU: XZZX surface codes under biased noise (p_Z = 2p/3, p_X = p_Y = p/6), the
paper's biased-noise experiment under parallel scheduling, against the oracle:
non-uniform Pauli priors, biased sampler thresholds, decisions and LER."""
import sys

import numpy as np
import pytest

import qecgen
from oracle import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2407_11523_amd as P  # noqa: E402


def np_(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("L,p,variant,alpha", [(5, 0.10, "ewainit", 0.5), (7, 0.10, "ewainit", 0.5),
                                               (9, 0.08, "bp", 1.0)])
def test_biased_xzzx_vs_oracle(L, p, variant, alpha):
    code = qecgen.xzzx(L)
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    probs = qecgen.biased_probs(code.n, p)
    thr = qecgen.thresholds(*probs[0])
    shots = 4000
    err, syn = P.sample(g, shots, thr, seed=31 + L)
    e_o, s_o = O.sample(code.hx, code.hz, shots, thr, seed=31 + L)
    assert np.array_equal(np_(syn), s_o) and np.array_equal(np_(err), e_o)
    r = P.decode(g, P.Params(variant=variant, alpha=alpha, max_iter=100), P.prior_llr(probs), syn)
    _, cnt = P.bookkeep(g, err, r["est"])
    torch.cuda.synchronize()
    ro = O.decode(code.hx, code.hz, O.Params(variant=variant, alpha=alpha, max_iter=100), O.prior_llr(probs), s_o)
    _, co = O.bookkeep(code.hx, code.hz, code.lx, code.lz, e_o, ro["est"])
    both = np_(r["conv"]).astype(bool) & ro["conv"].astype(bool)
    agree = float((np_(r["est"]) == ro["est"])[both].mean())
    ler_g = int(cnt[1] + cnt[2]) / shots
    lo, hi = O.wilson_ci(int(co[1] + co[2]), shots, z=3.29)
    print("biased", L, p, variant, dict(agree=agree, ler_g=ler_g, ler_o=int(co[1] + co[2]) / shots, ci=(lo, hi)),
          flush=True)
    sys.stdout.flush()
    assert agree >= 0.999
    assert lo <= ler_g <= hi
