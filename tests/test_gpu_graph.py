"""GPU: decodes captured as HIP graphs and replayed.

Each test captures library calls once, then, several times, writes new
syndromes into the captured input buffers eagerly (with other eager work in
between), replays the graph, and checks every replay against an eager decode of
the same syndromes, bit for bit.
"""
import sys

import pytest

import qecgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2407_11523_amd as P  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_mixed_step_graph_replays_match_eager():
    codes = [qecgen.planar(5), qecgen.toric(6), qecgen.xzzx(9)]
    shots = [3000, 2000, 1000]
    p = 0.08
    thr = qecgen.thresholds(p / 3, p / 3, p / 3)
    prm = P.Params(variant="ewainit", alpha=0.5, max_iter=60)
    items = []
    for c, s in zip(codes, shots):
        g = P.Graph(c.hx, c.hz, c.lx, c.lz)
        err = torch.empty((s, c.n), dtype=torch.uint8, device="cuda")
        syn = torch.empty((s, c.m), dtype=torch.uint8, device="cuda")
        counts = torch.zeros(3, dtype=torch.int64, device="cuda")
        items.append(dict(g=g, err=err, syn=syn, counts=counts, prior=P.prior_llr(qecgen.depolarizing_probs(c.n, p))))
    for it in items:
        P.sample(it["g"], it["syn"].shape[0], thr, 1, err=it["err"], synd=it["syn"])
    batch = P.MixedBatch([(it["g"], prm, it["prior"], it["syn"], 0) for it in items])

    def step():
        batch.run()
        for it, o in zip(items, batch.outs):
            it["counts"].zero_()
            P.bookkeep(it["g"], it["err"], o["est"], counts=it["counts"])

    cap = P.Captured(step)
    for rep, seed in enumerate((11, 12, 13)):
        for it in items:                       # new inputs, eagerly
            P.sample(it["g"], it["syn"].shape[0], thr, seed, err=it["err"], synd=it["syn"])
        torch.cuda.synchronize()
        cap.replay()
        torch.cuda.synchronize()
        got = [(o["est"].clone(), o["iters"].clone(), it["counts"].clone()) for it, o in zip(items, batch.outs)]
        for it, (est, iters, counts) in zip(items, got):   # eager reference of the same syndromes
            r = P.decode(it["g"], prm, it["prior"], it["syn"])
            _, cnt = P.bookkeep(it["g"], it["err"], r["est"])
            torch.cuda.synchronize()
            assert torch.equal(est, r["est"]) and torch.equal(iters, r["iters"]), rep
            assert torch.equal(counts, cnt), rep
        say("mixed replay", rep, [int(c[2].sum()) for c in got])


def test_soa_iteration_block_graph_replays_match_eager():
    c = qecgen.planar(13)
    g = P.Graph(c.hx, c.hz, c.lx, c.lz)
    shots = 5000
    p = 0.1
    thr = qecgen.thresholds(p / 3, p / 3, p / 3)
    prm = P.Params(variant="momentum", alpha=0.6, gamma=0.2, max_iter=40)
    pr = P.prior_llr(qecgen.depolarizing_probs(c.n, p))
    err = torch.empty((shots, c.n), dtype=torch.uint8, device="cuda")
    syn = torch.empty((shots, c.m), dtype=torch.uint8, device="cuda")
    P.sample(g, shots, thr, 5, err=err, synd=syn)
    out = {"est": torch.empty((shots, c.n), dtype=torch.uint8, device="cuda"),
           "conv": torch.empty(shots, dtype=torch.uint8, device="cuda"),
           "iters": torch.empty(shots, dtype=torch.int32, device="cuda")}
    ws = torch.empty(g.soa_workspace_bytes(prm, shots, 2048), dtype=torch.uint8, device="cuda")

    def run():
        return P.decode(g, prm, pr, syn, kernel="soa", soa_lanes=2048, soa_iter_block=6, out=out, ws=ws)

    cap = P.Captured(run)
    for rep, seed in enumerate((21, 22, 23)):
        P.sample(g, shots, thr, seed, err=err, synd=syn)
        other = P.decode(g, prm, pr, syn[:100])            # unrelated eager work between replays
        torch.cuda.synchronize()
        cap.replay()
        torch.cuda.synchronize()
        got = {k: v.clone() for k, v in out.items()}
        r = P.decode(g, prm, pr, syn)
        torch.cuda.synchronize()
        for k in ("est", "conv", "iters"):
            assert torch.equal(got[k], r[k]), (rep, k)
        assert torch.equal(other["iters"], r["iters"][:100])
        say("soa replay", rep, float(got["iters"].float().mean()))


def test_unrolled_forward_backward_graph_replays_match_eager():
    """The unrolled forward and its adjoint (two kernels per checkpoint segment plus
    the reductions) captured once; each replay's loss and gradients equal an eager
    autograd pass over the same shots bit for bit."""
    import ctypes

    import numpy as np
    from paper_2407_11523_amd import api as A
    c = qecgen.planar(5)
    T, K, shots, p = 10, 3, 1000, 0.08
    g = P.Graph(c.hx, c.hz, c.lx, c.lz)
    thr = qecgen.thresholds(p / 3, p / 3, p / 3)
    rng = np.random.default_rng(3)
    alpha = torch.tensor(rng.uniform(0.3, 0.9, T), dtype=torch.float32, device="cuda")
    prior = torch.tensor(np.log((1 - p) / (p / 3)) + rng.uniform(-0.3, 0.3, (c.n, 3)), dtype=torch.float32,
                         device="cuda")
    err = torch.empty((shots, c.n), dtype=torch.uint8, device="cuda")
    syn = torch.empty((shots, c.m), dtype=torch.uint8, device="cuda")
    sb, wb = A.unrolled_sizes(g, T, K, shots)
    saved = torch.empty(sb, dtype=torch.uint8, device="cuda")
    ws = torch.empty(wb, dtype=torch.uint8, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    dl = torch.ones(1, dtype=torch.float32, device="cuda")
    dalpha = torch.empty(T, dtype=torch.float64, device="cuda")
    dprior = torch.empty(c.n, 3, dtype=torch.float64, device="cuda")
    lib = g._lib

    def run():
        s = A._stream(syn.device)
        A.check(lib.bp4_unrolled_forward(g.handle, A._ptr(g.dev), 3, T, K, 30.0, shots, A._ptr(alpha), A._ptr(prior),
                                         A._ptr(syn), A._ptr(err), A._ptr(loss), ctypes.c_void_p(0), A._ptr(saved),
                                         sb, A._ptr(ws), wb, s))
        A.check(lib.bp4_unrolled_backward(g.handle, A._ptr(g.dev), 3, T, K, 30.0, shots, A._ptr(alpha), A._ptr(prior),
                                          A._ptr(syn), A._ptr(err), A._ptr(dl), A._ptr(saved), sb, A._ptr(dalpha),
                                          A._ptr(dprior), A._ptr(ws), wb, s))

    P.sample(g, shots, thr, 30, err=err, synd=syn)
    cap = P.Captured(run)
    for rep, seed in enumerate((31, 32, 33)):
        P.sample(g, shots, thr, seed, err=err, synd=syn)
        P.decode(g, P.Params(), prior, syn[:100])        # unrelated eager work between replays
        torch.cuda.synchronize()
        cap.replay()
        torch.cuda.synchronize()
        got = (loss.clone(), dalpha.clone(), dprior.clone())
        a = alpha.clone().requires_grad_(True)
        pr = prior.clone().requires_grad_(True)
        ref = P.unrolled_loss(g, a, pr, syn, err, T, K)
        ref.backward()
        torch.cuda.synchronize()
        assert torch.equal(got[0][0], ref.detach()), rep
        assert torch.equal(got[1].to(torch.float32), a.grad), rep
        assert torch.equal(got[2].to(torch.float32), pr.grad), rep
        say("unrolled replay", rep, float(got[0][0]))
