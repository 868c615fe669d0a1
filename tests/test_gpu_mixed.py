"""GPU: the persistent mixed-code launch and the per-phase plain decoder.

Both run the same per-node arithmetic as the single-code LDS kernel, so their
outputs must be bit-identical to it; the mixed batch is also checked against
the FP64 oracle on a sample of every code.
"""
import sys

import numpy as np
import pytest

import qecgen
from oracle import oracle as O
from qecgen import configs
from tests import bars

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


def setup(code, p, shots, seed):
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    thr = qecgen.thresholds(p / 3, p / 3, p / 3)
    err, syn = P.sample(g, shots, thr, seed=seed)
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p))
    return g, err, syn, pr


@pytest.mark.parametrize("make,variant,alpha", [(lambda: qecgen.planar(5), "ewainit", 0.5),
                                                (lambda: qecgen.toric(6), "bp", 1.0),
                                                (lambda: qecgen.xzzx(5), "momentum", 0.6),
                                                (lambda: qecgen.planar(7), "adagrad", 5.0)])
def test_plain_equals_lds_bitwise(make, variant, alpha):
    code = make()
    g, err, syn, pr = setup(code, 0.08, 20000, 41)
    prm = P.Params(variant=variant, alpha=alpha, max_iter=60)
    a = P.decode(g, prm, pr, syn)
    b = P.decode_plain(g, prm, pr, syn)
    torch.cuda.synchronize()
    say("plain", code.name, variant, b["iterations_run"], float(a["iters"].float().mean()))
    for k in ("est", "conv", "iters"):
        assert torch.equal(a[k], b[k]), k
    assert b["iterations_run"] == int(a["iters"].max())


CONFIG3 = list(configs.CONFIG3_CODES)
ALPHA3 = configs.alpha(3, "ewainit")


def test_mixed_equals_per_code_bitwise():
    # all config-3 codes in one launch (shots scaled down), mixed variants and group sizes
    variants = [("ewainit", 0.5), ("bp", 1.0), ("momentum", 0.6), ("adagrad", 5.0)]
    entries, ref = [], []
    for i, (fam, L, mult) in enumerate(CONFIG3):
        code = qecgen.make(fam, L)
        g, err, syn, pr = setup(code, 0.08, 2048 * mult + 37 * i, 50 + i)
        variant, alpha = variants[i % 4]
        prm = P.Params(variant=variant, alpha=alpha, max_iter=100)
        lanes = [0, 64, 32, 16, 8, 128, 256][i % 7]
        try:
            r = P.decode(g, prm, pr, syn, group_lanes=lanes)
        except P.BP4Error:          # this group size does not fit the code (lanes or LDS)
            lanes = 0
            r = P.decode(g, prm, pr, syn)
        entries.append((g, prm, pr, syn, lanes))
        ref.append(r)
    outs = P.decode_mixed(entries)
    torch.cuda.synchronize()
    for (fam, L, _), o, r in zip(CONFIG3, outs, ref):
        for k in ("est", "conv", "iters"):
            assert torch.equal(o[k], r[k]), (fam, L, k)


def test_mixed_matches_oracle_sample():
    entries, codes, errs = [], [], []
    for i, (fam, L, mult) in enumerate(CONFIG3):
        code = qecgen.make(fam, L)
        g, err, syn, pr = setup(code, 0.08, 4096 * mult, qecgen.config_seed(3, i, 0))
        entries.append((g, P.Params(variant="ewainit", alpha=ALPHA3, max_iter=100), pr, syn, 0))
        codes.append(code)
        errs.append(err)
    outs = P.decode_mixed(entries)
    torch.cuda.synchronize()
    for i, (code, o) in enumerate(zip(codes, outs)):
        k = 1024
        e_o, s_o = O.sample(code.hx, code.hz, k, qecgen.thresholds(0.08 / 3, 0.08 / 3, 0.08 / 3),
                            seed=qecgen.config_seed(3, i, 0))
        assert np.array_equal(np_(entries[i][3][:k]), s_o)
        op = O.Params(variant="ewainit", alpha=ALPHA3, max_iter=100)
        bar = bars.decision_bar(code, op, O.prior_llr(qecgen.depolarizing_probs(code.n, 0.08)), s_o,
                                np_(o["est"][:k]))
        ro = bar.pop("ro")
        bar.pop("rp")
        bars.early_exact(np_(o["est"][:k]), np_(o["conv"][:k]), np_(o["iters"][:k]), ro)
        _, cg = P.bookkeep(entries[i][0], errs[i], o["est"])
        _, co = O.bookkeep(code.hx, code.hz, code.lx, code.lz, e_o, ro["est"])
        torch.cuda.synchronize()
        ler_g = int(cg[1] + cg[2]) / errs[i].shape[0]
        lo, hi = O.wilson_ci(int(co[1] + co[2]), k, z=3.29)
        say("mixed-vs-oracle", code.name, bar, ler_g, (lo, hi))
        # Non-converged shots run iter_max chaotic iterations, where the FP64 oracle does not
        # agree with itself under a 1e-7 relative prior perturbation: the bar is measured.
        assert bar["ok"], (code.name, bar)
        assert lo <= ler_g <= hi


def test_mixed_full_batch_in_bench_launch():
    """The full mixed batch (26 x 2^18 = 6,815,744 shots over the 11 codes, p = 0.08,
    EWAInit with the chosen discount, iter_max 100) in the launch the benchmark
    times: the lane mappings from the committed autotuner cache, one persistent
    launch over every code.  128 shots per code (the first two, the last, 125 drawn
    at random) are decoded by the oracle from its own sampler's rows.

    Bar, over the 1,408 sampled shots: the decisions agree at least as well as the
    oracle agrees with itself under a 1e-7 relative prior perturbation, minus a
    3-sigma margin, or 99.9% where that is lower; shots the oracle stops within 20
    iterations agree exactly, and so do their stopping iterations except where the
    FP64 hard decision at the earlier one was within 1e-3 (relative) of a tie, on at
    most 1% of them; each code's logical error rate over its whole batch lies in the
    oracle's 99.9% interval on its sample."""
    from paper_2407_11523_amd import tune
    from tests.oracle_inputs import matched
    p = 0.08
    thr = qecgen.thresholds(p / 3, p / 3, p / 3)
    prm = P.Params(variant="ewainit", alpha=ALPHA3, max_iter=100)
    op = O.Params(variant="ewainit", alpha=ALPHA3, max_iter=100)
    items = []
    for i, (fam, L, mult) in enumerate(CONFIG3):
        code = qecgen.make(fam, L)
        shots = (1 << 18) * mult
        g = P.Graph(code.hx, code.hz, code.lx, code.lz)
        err, syn = P.sample(g, shots, thr, seed=qecgen.config_seed(3, i, 0))
        items.append(dict(code=code, g=g, err=err, syn=syn, shots=shots, seed=qecgen.config_seed(3, i, 0),
                          prior=P.prior_llr(qecgen.depolarizing_probs(code.n, p))))
    tuned = tune.tune_mixed([(it["g"], prm, it["prior"], it["syn"]) for it in items],
                            [tune.digest(it["code"].hx, it["code"].hz) for it in items],
                            [it["shots"] for it in items], save=False)
    say("full mixed batch lanes", tuned["lanes"], "cached" if tuned.get("cached") else "measured")
    batch = P.MixedBatch([(it["g"], prm, it["prior"], it["syn"], G) for it, G in zip(items, tuned["lanes"])])
    batch.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    d_gpu, d_self, n_off, n_early = [], [], 0, 0
    for it, o in zip(items, batch.outs):
        code, shots = it["code"], it["shots"]
        idx = np.unique(np.concatenate([[0, 1, shots - 1], rng.choice(shots, 125, replace=False)]))
        e_o, s_o = matched(code, thr, it["seed"], it["err"], it["syn"], idx=idx)
        pi = O.prior_llr(qecgen.depolarizing_probs(code.n, p))
        sel = torch.as_tensor(idx, device=it["syn"].device)
        est_g, conv_g, it_g = np_(o["est"][sel]), np_(o["conv"][sel]), np_(o["iters"][sel])
        ro = O.decode(code.hx, code.hz, op, pi, s_o)
        rp = O.decode(code.hx, code.hz, op, bars.perturbed_prior(pi), s_o)
        d_gpu.append((est_g != ro["est"]).mean(axis=1))
        d_self.append((rp["est"] != ro["est"]).mean(axis=1))
        early = bars.early_exact(est_g, conv_g, it_g, ro)
        # a stopping iteration may differ only where the FP64 decision was a near-tie
        off, margins = bars.same_stops(code, op, pi, s_o[early], it_g[early], ro["iters"][early])
        n_off += len(off)
        n_early += int(early.sum())
        _, cg = P.bookkeep(it["g"], it["err"], o["est"])
        _, co = O.bookkeep(code.hx, code.hz, code.lx, code.lz, e_o, ro["est"])
        torch.cuda.synchronize()
        ler_g = int(cg[1] + cg[2]) / shots
        lo, hi = O.wilson_ci(int(co[1] + co[2]), len(idx), z=3.29)
        say("full mixed batch", code.name, shots, dict(early=int(early.sum()), stop_diff=len(off), margins=margins,
                                                       gpu=1 - float(d_gpu[-1].mean()),
                                                       self=1 - float(d_self[-1].mean()), ler_g=ler_g, ci=(lo, hi)))
        assert lo <= ler_g <= hi, code.name
    d_gpu, d_self = np.concatenate(d_gpu), np.concatenate(d_self)
    gpu, self_ = 1 - float(d_gpu.mean()), 1 - float(d_self.mean())
    margin = bars.Z_MARGIN * float(np.sqrt(d_gpu.var() / len(d_gpu) + d_self.var() / len(d_self)))
    bar = min(bars.TARGET, self_ - margin)
    say("full mixed batch agreement", dict(gpu=gpu, self=self_, margin=margin, bar=bar), "stops differing", n_off,
        n_early)
    assert gpu >= bar
    assert n_off <= max(2, 0.01 * n_early)


def test_mixed_edge_cases():
    c1, c2 = qecgen.toric(4), qecgen.planar(3)
    g1, _, s1, p1 = setup(c1, 0.05, 100, 1)
    g2, _, s2, p2 = setup(c2, 0.05, 0, 2)
    out = P.decode_mixed([(g1, P.Params(), p1, s1, 0), (g2, P.Params(), p2, s2, 0)])
    torch.cuda.synchronize()
    ref = P.decode(g1, P.Params(), p1, s1)
    torch.cuda.synchronize()
    assert torch.equal(out[0]["est"], ref["est"]) and out[1]["est"].shape == (0, c2.n)
    with pytest.raises(P.BP4Error):
        P.decode_mixed([])


def test_group_size_does_not_change_results():
    # every lane-group size runs the same per-node arithmetic: outputs are bit-identical
    code = qecgen.planar(9)
    g, err, syn, pr = setup(code, 0.08, 5000, 61)
    for variant, alpha in (("ewainit", 0.5), ("adagrad", 5.0)):
        prm = P.Params(variant=variant, alpha=alpha, max_iter=100)
        ref = P.decode(g, prm, pr, syn, group_lanes=64)
        for G in (8, 16, 32, 128, 256):
            try:
                r = P.decode(g, prm, pr, syn, group_lanes=G, lds_bytes=40960)
            except P.BP4Error:
                continue
            torch.cuda.synchronize()
            for k in ("est", "conv", "iters"):
                assert torch.equal(r[k], ref[k]), (variant, G, k)


def test_autotuner_picks_feasible_sizes(tmp_path):
    from paper_2407_11523_amd import tune
    entries, digests, shots = [], [], []
    for fam, L in (("planar", 5), ("toric", 10)):
        code = qecgen.make(fam, L)
        g, err, syn, pr = setup(code, 0.08, 4096, 71)
        entries.append((g, P.Params(variant="ewainit", alpha=0.5), pr, syn))
        digests.append(tune.digest(code.hx, code.hz))
        shots.append(1 << 18)
    res = tune.tune_mixed(entries, digests, shots, sample=2048, cache_path=str(tmp_path / "c.json"))
    say("tuned", res["lanes"], res["budget"])
    for (g, p, _, _), (G, S) in zip(entries, res["lanes"]):
        assert (G in tune.GROUP_SIZES and S == 0) or (G == 0 and S >= 1)
        assert tune.layout_bytes(g, p, G, S) <= res["budget"]
    again = tune.tune_mixed(entries, digests, shots, sample=2048, cache_path=str(tmp_path / "c.json"))
    assert again["lanes"] == res["lanes"]
