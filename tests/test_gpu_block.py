"""GPU: block slots of the LDS kernel (S shots sharing the 512 lanes of a workgroup,
which walk the flattened (slot, check) and (slot, qubit) items).

The per-node arithmetic is the wave groups' own, so every slot count must give
bit-identical decisions, convergence flags, iteration counts and final states
(posteriors and both message directions) to a wave-group decode, for every
variant, with ragged shot counts (not a multiple of S, fewer shots than slots)
and inside a mixed launch.
"""
import sys

import numpy as np
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


def clifford_relabel(code, seed):
    rng = np.random.default_rng(seed)
    lab = code.labels()
    new = np.zeros_like(lab)
    for v in range(code.n):
        p = rng.permutation([1, 2, 3])
        mp = np.array([0, p[0], p[1], p[2]], np.uint8)
        new[:, v] = mp[lab[:, v]]
    return (new & 1).astype(np.uint8), (new >> 1).astype(np.uint8)


def setup(hx, hz, lx, lz, p, shots, seed):
    g = P.Graph(hx, hz, lx, lz)
    err, syn = P.sample(g, shots, qecgen.thresholds(p / 3, p / 3, p / 3), seed=seed)
    pr = P.prior_llr(qecgen.depolarizing_probs(g.n, p))
    return g, syn, pr


VARIANTS = [("ewainit", dict(alpha=0.5)), ("bp", dict()), ("momentum", dict(alpha=0.6, gamma=0.3)),
            ("adagrad", dict(alpha=5.0)), ("aewa", dict(alpha=1.0, alpha_last=0.0, alpha_steps=4, max_iter=12))]


@pytest.mark.parametrize("variant,kw", VARIANTS, ids=[v for v, _ in VARIANTS])
def test_block_slots_equal_wave_groups(variant, kw):
    c = qecgen.planar(9)
    g, syn, pr = setup(c.hx, c.hz, c.lx, c.lz, 0.09, 3001, 7)
    prm = P.Params(variant=variant, **dict(dict(max_iter=60), **kw))
    ref = P.decode(g, prm, pr, syn, group_lanes=32)
    for S in (1, 2, 3, 5, 7, 16):
        try:
            r = P.decode(g, prm, pr, syn, block_shots=S, lds_bytes=0)
        except P.BP4Error:          # the S slots do not fit the LDS
            say("skip", S)
            continue
        torch.cuda.synchronize()
        for k in ("est", "conv", "iters"):
            assert torch.equal(r[k], ref[k]), (variant, S, k)
    say("block", variant, float(ref["iters"].float().mean()), int(ref["conv"].sum()))


@pytest.mark.parametrize("name", ["toric6", "xzzx5-clifford"])
def test_block_slot_states_bitwise(name):
    if name == "toric6":
        c = qecgen.toric(6)
        hx, hz = c.hx, c.hz
    else:
        c = qecgen.xzzx(5)
        hx, hz = clifford_relabel(c, 3)
    g, syn, pr = setup(hx, hz, c.lx, c.lz, 0.1, 997, 11)
    for variant, kw in VARIANTS[:4]:
        prm = P.Params(variant=variant, max_iter=5, stop_on_syndrome=False, **kw)
        ref = P.decode(g, prm, pr, syn, trace=True, group_lanes=16)
        for S in (3, 11):
            r = P.decode(g, prm, pr, syn, trace=True, block_shots=S)
            torch.cuda.synchronize()
            for k in ("est", "conv", "iters", "q", "mvc", "mcv"):
                assert torch.equal(r[k], ref[k]), (name, variant, S, k)


def test_block_slot_ragged_shot_counts():
    c = qecgen.toric(4)
    prm = P.Params(variant="ewainit", alpha=0.5, max_iter=40)
    for shots, S in ((1, 8), (3, 8), (9, 8), (65, 4), (257, 32)):
        g, syn, pr = setup(c.hx, c.hz, c.lx, c.lz, 0.12, shots, 100 + shots)
        ref = P.decode(g, prm, pr, syn, group_lanes=8)
        r = P.decode(g, prm, pr, syn, block_shots=S)
        torch.cuda.synchronize()
        for k in ("est", "conv", "iters"):
            assert torch.equal(r[k], ref[k]), (shots, S, k)


def test_mixed_launch_with_block_slots():
    entries, ref = [], []
    specs = [(qecgen.planar(11), (0, 2)), (qecgen.toric(6), (0, 5)), (qecgen.xzzx(5), (32, 0)),
             (qecgen.planar(5), (0, 9)), (qecgen.toric(10), (256, 0))]
    for i, (c, (G, S)) in enumerate(specs):
        g, syn, pr = setup(c.hx, c.hz, c.lx, c.lz, 0.08, 2000 + 111 * i, 300 + i)
        prm = P.Params(variant=["ewainit", "momentum", "bp", "aewa", "adagrad"][i],
                       alpha=[0.5, 0.6, 1.0, 1.0, 5.0][i], max_iter=50)
        entries.append((g, prm, pr, syn, (G, S)))
        ref.append(P.decode(g, prm, pr, syn, group_lanes=G, block_shots=S))
    outs = P.decode_mixed(entries)
    torch.cuda.synchronize()
    for i, (o, r) in enumerate(zip(outs, ref)):
        for k in ("est", "conv", "iters"):
            assert torch.equal(o[k], r[k]), (i, k)


@pytest.mark.parametrize("variant,kw", [("ewainit", dict(alpha=0.5)),
                                        ("aewa", dict(alpha=1.0, alpha_last=0.0, alpha_steps=4, max_iter=30))])
def test_compacted_slots_keep_their_state(variant, kw):
    """Once the queue is empty, a slot left without a shot takes the region of the
    last active slot.  With early stopping the shots end at different iterations,
    so shots still running are moved mid-decode; their final messages and
    posteriors (traced after their last iteration) equal a wave-group decode bit for
    bit.  24 slots per workgroup and 1,500 shots: most of the decode is tail."""
    c = qecgen.planar(7)
    g, syn, pr = setup(c.hx, c.hz, c.lx, c.lz, 0.12, 1500, 29)
    prm = P.Params(variant=variant, **dict(dict(max_iter=60), **kw))
    ref = P.decode(g, prm, pr, syn, group_lanes=16, trace=True)
    r = P.decode(g, prm, pr, syn, block_shots=24, trace=True)
    torch.cuda.synchronize()
    say("compacted slots", variant, float(r["iters"].float().mean()), int(r["iters"].max()))
    assert int(r["iters"].max()) > 2 * int(r["iters"].min())   # shots end at different iterations
    for k in ("est", "conv", "iters", "q", "mvc", "mcv"):
        assert torch.equal(r[k], ref[k]), (variant, k)
