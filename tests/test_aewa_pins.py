"""AEWA-BP in the oracle (appendix on adaptive MBP): EWAInit-BP restarted with the
next discount of a list, largest first, until the syndrome is met.

Pinned by composition: the oracle's AEWA output must equal, shot by shot, what
separate EWAInit decodes with each discount give (the first one that converges,
or the last), with the iteration count summed over the attempts; EWAInit itself
is pinned elsewhere.  A single step is EWAInit; alpha = 1 is traditional BP.
"""
import numpy as np
import pytest

import qecgen
from oracle import oracle as O


def _case(make, p, shots, seed):
    code = make()
    e, s = O.sample(code.hx, code.hz, shots, qecgen.thresholds(p / 3, p / 3, p / 3), seed=seed)
    return code, e, s, O.prior_llr(qecgen.depolarizing_probs(code.n, p))


@pytest.mark.parametrize("make,p,lo,steps", [(lambda: qecgen.planar(5), 0.12, 0.0, 11),
                                             (lambda: qecgen.toric(4), 0.14, 0.5, 6),
                                             (lambda: qecgen.xzzx(5), 0.15, 0.2, 4)])
def test_aewa_is_the_first_converging_ewainit(make, p, lo, steps):
    code, e, s, pi = _case(make, p, 600, 4)
    T = 30
    ra = O.decode(code.hx, code.hz, O.Params(variant="aewa", alpha=1.0, alpha_last=lo, alpha_steps=steps,
                                             max_iter=T), pi, s)
    alphas = [1.0 + (lo - 1.0) * k / (steps - 1) for k in range(steps)]
    runs = [O.decode(code.hx, code.hz, O.Params(variant="ewainit", alpha=a, max_iter=T), pi, s) for a in alphas]
    restarted = 0
    for i in range(len(s)):
        k = next((k for k, r in enumerate(runs) if r["conv"][i]), steps - 1)
        assert np.array_equal(ra["est"][i], runs[k]["est"][i]), i
        assert ra["conv"][i] == runs[k]["conv"][i]
        assert ra["iters"][i] == k * T + runs[k]["iters"][i]
        restarted += k > 0
    assert restarted > 0          # the case exercises restarts
    # alpha = 1 as the first attempt is traditional BP
    rb = O.decode(code.hx, code.hz, O.Params(variant="bp", max_iter=T), pi, s)
    assert np.array_equal(runs[0]["est"], rb["est"]) and np.array_equal(runs[0]["iters"], rb["iters"])


def test_aewa_single_step_is_ewainit_and_needs_stopping():
    code, e, s, pi = _case(lambda: qecgen.planar(3), 0.1, 300, 9)
    a = O.decode(code.hx, code.hz, O.Params(variant="aewa", alpha=0.6, alpha_steps=1, max_iter=20), pi, s)
    b = O.decode(code.hx, code.hz, O.Params(variant="ewainit", alpha=0.6, max_iter=20), pi, s)
    for k in ("est", "conv", "iters"):
        assert np.array_equal(a[k], b[k])
    with pytest.raises(ValueError):
        O.decode(code.hx, code.hz, O.Params(variant="aewa", stop_on_syndrome=False, max_iter=5), pi, s)
    with pytest.raises(ValueError):
        O.decode(code.hx, code.hz, O.Params(variant="aewa", alpha_steps=0, max_iter=5), pi, s)
