"""GPU: the single-pass HBM kernel for large codes.

It evaluates the same per-node arithmetic in the same order as the two-phase
kernels (a qubit gathers its checks' other stored words phi(|m|) and sums them in
value order, exactly as the check pass sums them), so its hard decisions,
convergence flags and iteration counts must equal the SOA kernel's (and on codes
both run, the LDS kernel's) bit for bit, for every variant, shot count, workgroup
shape and stopping rule.  The oracle bar on the full large-code batch is in
test_gpu_soa.py (test_large_codes_full_batch_sampled, run for both HBM kernels).
"""
import sys

import pytest

import qecgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2407_11523_amd as P  # noqa: E402

# AEWA: the default attempt list, discounts 1, 0.9, ..., 0 (attempt k restarts from the priors)
VARIANTS = [("bp", 1.0, 0.0), ("ewainit", 0.6, 0.0), ("momentum", 0.6, 0.3), ("adagrad", 5.0, 0.0),
            ("aewa", 1.0, 0.0)]
CODES = [("planar", 5), ("xzzx", 9), ("toric", 8), ("planar", 31), ("toric", 32)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(g, prm, pr, syn, kernel, **kw):
    r = P.decode(g, prm, pr, syn, kernel=kernel, **kw)
    torch.cuda.synchronize()
    return r


def same(a, b, what, n=None):
    """Outputs equal bit for bit (on the first n shots of a, if given)."""
    for k in ("est", "conv", "iters"):
        x = a[k] if n is None else a[k][:n]
        assert torch.equal(x, b[k]), (what, k, int((x != b[k]).sum()))


@pytest.mark.parametrize("fam,size", CODES)
@pytest.mark.parametrize("variant,alpha,gamma", VARIANTS)
def test_gather_equals_two_phase(fam, size, variant, alpha, gamma):
    code = qecgen.make(fam, size)
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    p = 0.10
    shots = 4100 if size > 20 else 5000
    _, syn = P.sample(g, shots, qecgen.thresholds(p / 3, p / 3, p / 3), seed=size * 31 + len(variant))
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p))
    prm = P.Params(variant=variant, alpha=alpha, gamma=gamma, max_iter=60)
    say("gather vs soa", code.name, variant, shots)
    ref = run(g, prm, pr, syn, "soa")
    r = run(g, prm, pr, syn, "gather")
    same(ref, r, (code.name, variant, "soa"))
    if size <= 20:
        same(run(g, prm, pr, syn, "lds"), r, (code.name, variant, "lds"))
    say("  conv", float(r["conv"].float().mean()), "iters", float(r["iters"].float().mean()))


@pytest.mark.parametrize("fam,size", [("planar", 31), ("toric", 32), ("xzzx", 9)])
def test_gather_walk_order_changes_nothing(fam, size):
    """The walk order is a locality choice only: the lattice-strip walk that qubit
    coordinates select, and the one a random layout selects, give the same outputs
    as the default walk and the two-phase kernel, across a queue tail long enough for
    the live shots to move to the lower columns."""
    code = qecgen.make(fam, size)
    p = 0.10
    plain = P.Graph(code.hx, code.hz, code.lx, code.lz)
    lattice = P.Graph(code.hx, code.hz, code.lx, code.lz, coords=code.coords)
    rng = torch.Generator().manual_seed(size)
    rand_xy = torch.randint(-1000, 1000, (code.n, 2), generator=rng, dtype=torch.int32).numpy()
    scrambled = P.Graph(code.hx, code.hz, code.lx, code.lz, coords=rand_xy)
    shots = 9000
    _, syn = P.sample(plain, shots, qecgen.thresholds(p / 3, p / 3, p / 3), seed=size + 100)
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p))
    for variant, alpha, gamma in (("ewainit", 0.6, 0.0), ("momentum", 0.6, 0.3), ("aewa", 1.0, 0.0)):
        prm = P.Params(variant=variant, alpha=alpha, gamma=gamma, max_iter=70)
        say("walk orders", code.name, variant)
        ref = run(plain, prm, pr, syn, "soa")
        same(ref, run(plain, prm, pr, syn, "gather"), (code.name, variant, "default walk"))
        same(ref, run(lattice, prm, pr, syn, "gather"), (code.name, variant, "lattice strips"))
        same(ref, run(scrambled, prm, pr, syn, "gather"), (code.name, variant, "random layout"))


def test_gather_shot_counts_and_shapes():
    """Fewer shots than one workgroup, ragged counts, more shots than columns in flight
    (lanes take new shots in place), and 4, 8 or 16 wavefronts per workgroup."""
    code = qecgen.planar(9)
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    p = 0.12
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p))
    prm = P.Params(variant="ewainit", alpha=0.6, max_iter=80)
    for shots in (1, 63, 64, 65, 20000):
        _, syn = P.sample(g, shots, qecgen.thresholds(p / 3, p / 3, p / 3), seed=shots + 5)
        ref = run(g, prm, pr, syn, "soa")
        for waves in (4, 8, 16):
            say("gather shots", shots, "waves", waves)
            same(ref, run(g, prm, pr, syn, "gather", gather_waves=waves), (shots, waves))
    # more shots than the 16,384 columns of a full chip: every lane is refilled many times
    shots = (1 << 16) + 77
    _, syn = P.sample(g, shots, qecgen.thresholds(p / 3, p / 3, p / 3), seed=3)
    say("gather shots", shots)
    same(run(g, prm, pr, syn, "soa"), run(g, prm, pr, syn, "gather"), shots)
    # zero shots: nothing launched
    z = torch.empty(0, code.m, dtype=torch.uint8, device="cuda")
    assert run(g, prm, pr, z, "gather")["est"].shape == (0, code.n)


def test_gather_stopping_rules():
    """No early stop (every shot runs max_iter, conv reports the last test), a single
    iteration, and a zero syndrome (converges at t = 1 when every prior is positive)."""
    code = qecgen.toric(10)
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    p = 0.08
    _, syn = P.sample(g, 3000, qecgen.thresholds(p / 3, p / 3, p / 3), seed=11)
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p))
    for prm in (P.Params(variant="ewainit", alpha=0.6, max_iter=7, stop_on_syndrome=False),
                P.Params(variant="adagrad", alpha=5.0, max_iter=9, stop_on_syndrome=False),
                P.Params(variant="momentum", alpha=0.6, gamma=0.7, max_iter=1),
                P.Params(variant="bp", max_iter=1)):
        say("gather stop rule", prm)
        r = run(g, prm, pr, syn, "gather")
        same(run(g, prm, pr, syn, "soa"), r, prm)
        if not prm.stop_on_syndrome:
            assert bool((r["iters"] == prm.max_iter).all())
    zero = torch.zeros(100, code.m, dtype=torch.uint8, device="cuda")
    r = run(g, P.Params(variant="ewainit", alpha=0.6, max_iter=20), pr, zero, "gather")
    assert bool((r["iters"] == 1).all()) and bool((r["conv"] == 1).all()) and int(r["est"].sum()) == 0


def test_gather_ignores_stale_workspace():
    """The records start with whatever the workspace holds: a fresh shot reads the
    initial messages from the table, never its record, so a workspace full of NaN
    bytes, or one left by another decode, gives the same results."""
    code = qecgen.planar(13)
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    p = 0.1
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p))
    prm = P.Params(variant="momentum", alpha=0.6, gamma=0.3, max_iter=50)
    _, syn = P.sample(g, 9000, qecgen.thresholds(p / 3, p / 3, p / 3), seed=21)
    _, syn2 = P.sample(g, 9000, qecgen.thresholds(p / 3, p / 3, p / 3), seed=22)
    ws = torch.full((g.gather_workspace_bytes(prm, 9000),), 0xFF, dtype=torch.uint8, device="cuda")
    a = run(g, prm, pr, syn, "gather", ws=ws)
    run(g, prm, pr, syn2, "gather", ws=ws)
    b = run(g, prm, pr, syn, "gather", ws=ws)
    same(a, b, "stale")
    same(run(g, prm, pr, syn, "soa"), a, "soa")


def test_auto_runs_gather_on_large_codes():
    """The automatic choice for a large decode is the single-pass kernel (the workspace it
    sizes is the single-pass one), AEWA and the serial schedule included; the verification
    outputs keep the SOA kernel, and the single-pass kernel refuses them."""
    code = qecgen.planar(31)
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    p = 0.1
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p))
    prm = P.Params(variant="ewainit", alpha=0.6, max_iter=40)
    assert g.workspace_bytes(prm, 5000) == g.gather_workspace_bytes(prm, 5000)
    _, syn = P.sample(g, 5000, qecgen.thresholds(p / 3, p / 3, p / 3), seed=8)
    same(run(g, prm, pr, syn, "gather"), run(g, prm, pr, syn, "auto"), "auto")
    tr = run(g, prm, pr, syn[:64], "auto", trace=True)
    same(run(g, prm, pr, syn[:64], "soa"), tr, "trace")
    with pytest.raises(P.BP4Error):
        P.decode(g, prm, pr, syn[:64], kernel="gather", trace=True)
    ser = P.Params(variant="ewainit", alpha=0.6, max_iter=20, serial=True)
    assert g.workspace_bytes(ser, 5000) == g.gather_workspace_bytes(ser, 5000)
    same(run(g, ser, pr, syn[:600], "gather"), run(g, ser, pr, syn[:600], "auto"), "auto serial")
    ae = P.Params(variant="aewa", alpha=1.0, alpha_last=0.0, alpha_steps=11, max_iter=30)
    assert g.workspace_bytes(ae, 5000) == g.gather_workspace_bytes(ae, 5000)
    same(run(g, ae, pr, syn, "gather"), run(g, ae, pr, syn, "auto"), "auto aewa")


def _clifford_relabel(code, seed):
    """Random local Clifford on every qubit: permutes each qubit's X, Y, Z labels, so
    the checks carry Y labels (the code stays a valid stabilizer code)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    lab = code.labels()
    new = np.zeros_like(lab)
    for v in range(code.n):
        p = rng.permutation([1, 2, 3])
        new[:, v] = np.array([0, p[0], p[1], p[2]], np.uint8)[lab[:, v]]
    return (new & 1).astype(np.uint8), (new >> 1).astype(np.uint8)


@pytest.mark.parametrize("variant,alpha,gamma", VARIANTS)
def test_gather_y_labels_and_per_qubit_priors(variant, alpha, gamma):
    """Y labels (a Clifford-relabelled toric code: three labels per qubit, the with-Y
    label sums and lambdas) and per-qubit priors (biased noise jittered per qubit, so the
    initial-message table differs from qubit to qubit): bit-identical to the two-phase
    kernel."""
    import numpy as np
    code = qecgen.toric(16)
    hx, hz = _clifford_relabel(code, 3)
    g = P.Graph(hx, hz)
    p = 0.09
    probs = qecgen.biased_probs(code.n, p) * np.random.default_rng(4).uniform(0.7, 1.3, (code.n, 1))
    pr = P.prior_llr(probs)
    _, syn = P.sample(g, 6000, qecgen.thresholds(p / 6, p / 6, 2 * p / 3), seed=9)
    prm = P.Params(variant=variant, alpha=alpha, gamma=gamma, max_iter=60)
    say("gather y labels", variant)
    same(run(g, prm, pr, syn, "soa"), run(g, prm, pr, syn, "gather"), variant)


def test_gather_aewa_attempts():
    """AEWA on the single-pass kernel: an unsolved shot keeps its column and restarts from
    the priors with the next discount (eq. EWAInit), its iterations summed over the
    attempts.  Short and long attempt lists, rising and falling discounts, several
    workgroup shapes, a batch where columns restart while others take new shots: equal
    to the LDS kernel's in-place restarts and the SOA kernel's attempt launches."""
    code = qecgen.planar(9)
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    p = 0.12
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p))
    _, syn = P.sample(g, 20000, qecgen.thresholds(p / 3, p / 3, p / 3), seed=41)
    for alpha, last, steps, mi in ((1.0, 0.0, 11, 25), (0.5, 0.9, 3, 10), (0.7, 0.7, 1, 40), (0.0, 1.0, 5, 3)):
        prm = P.Params(variant="aewa", alpha=alpha, alpha_last=last, alpha_steps=steps, max_iter=mi)
        ref = run(g, prm, pr, syn, "lds")
        assert int(ref["iters"].max()) > mi or steps == 1   # some shot restarted
        for waves in (4, 16):
            say("gather aewa", alpha, last, steps, mi, "waves", waves)
            same(ref, run(g, prm, pr, syn, "gather", gather_waves=waves), (alpha, last, steps, waves))
        same(ref, run(g, prm, pr, syn, "soa"), (alpha, last, steps, "soa"))


@pytest.mark.parametrize("variant,alpha,gamma", VARIANTS)
def test_gather_serial_schedule(variant, alpha, gamma):
    """The serial schedule (Algorithm 1) on the single-pass kernel: the level sweep with each
    column's record updated in place, a workgroup barrier after each level and, in a shot's
    first sweep, the words not yet rewritten taken from the initial table gives the
    qubit-by-qubit sweep bit for bit: equal to the LDS kernel's level sweep and the SOA
    kernel's one-lane sweep, for every variant, with Y labels, on a large code, for every
    workgroup shape and with lanes that take new shots while others run."""
    cases = [(qecgen.make("planar", 5), None), (qecgen.make("toric", 8), None), (qecgen.make("xzzx", 9), None),
             (qecgen.toric(6), 5)]
    for code, relabel in cases:
        hx, hz = (code.hx, code.hz) if relabel is None else _clifford_relabel(code, relabel)
        g = P.Graph(hx, hz)
        p = 0.09
        pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p))
        _, syn = P.sample(g, 3000, qecgen.thresholds(p / 3, p / 3, p / 3), seed=code.n + 3)
        prm = P.Params(variant=variant, alpha=alpha, gamma=gamma, max_iter=40, serial=True)
        say("gather serial", code.name, relabel, variant)
        ref = run(g, prm, pr, syn, "lds")
        same(ref, run(g, prm, pr, syn, "gather"), (code.name, variant))
        same(ref, run(g, prm, pr, syn, "gather", gather_waves=4), (code.name, variant, 4))
        same(ref, run(g, prm, pr, syn[:700], "soa"), (code.name, variant, "soa"), n=700)
    code = qecgen.planar(31)
    g = P.Graph(code.hx, code.hz, code.lx, code.lz)
    pr = P.prior_llr(qecgen.depolarizing_probs(code.n, 0.06))
    _, syn = P.sample(g, 1500, qecgen.thresholds(0.02, 0.02, 0.02), seed=61)
    prm = P.Params(variant=variant, alpha=alpha, gamma=gamma, max_iter=25, serial=True)
    say("gather serial planar 31", variant)
    same(run(g, prm, pr, syn, "soa"), run(g, prm, pr, syn, "gather"), ("planar31", variant))
