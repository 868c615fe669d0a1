#!/usr/bin/env python3
"""Throughput of the mixed-code persistent GF(4) BP decode on one MI355X.

Workload (one step): the mixed batch of planar d in {5,7,9,11,13}, toric L in
{6,10,14} and XZZX L in {5,9,13} surface codes under depolarizing noise
p = 0.08, 2^18 shots per code scaled 1:2:4 from the smallest to the largest
size of each family (26 x 2^18 = 6,815,744 shots), EWAInit-BP with iter_max
100.  A step samples every code's errors and syndromes on the GPU, decodes all
codes in one persistent launch, and classifies every shot (success, detected,
undetected).  Inputs are synthetic and seeded; nothing is read from disk.

Prints one JSON line.  Besides the contract fields it reports the per-code
plain decoder on the same syndromes (the reference point of the metric), the
decode kernel's fraction of its VALU roofline, and the FP64 CPU oracle timed on
a bounded sample of the same shots.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from qecgen import configs  # noqa: E402

P_ERR = configs.CONFIG3["p"]
ALPHA = configs.alpha(3, "ewainit")     # EWAInit discount of the mixed batch (chosen on the oracle)
ALPHA_EXTRA = 0.5    # the paper's trapping-set value, for the sections it gives no discount for
MOMENTUM_ALPHA = configs.alpha(2, "momentum")   # Momentum step of the toric sweep (chosen on the oracle)
MAX_ITER = configs.CONFIG3["max_iter"]
BASE_SHOTS = configs.CONFIG3["base_shots"]
# (family, size, shot multiplier): smallest size(s) 1, middle 2, largest 4
CODES = list(configs.CONFIG3_CODES)

# Roofline of the LDS-resident decode: VALU issue.  Algorithmic work of one flooding
# iteration of one shot, counted at the level of the update rules: per edge one tanh
# and one atanh for the check message and one exp and one log for lambda
# (4 transcendentals), per qubit 3 exponentials for the posterior's probabilities,
# and 15-20 plain FP32 operations per edge (leave-one-out products, posterior sums,
# extrinsic subtraction, lambda's arithmetic, the EWA update, the hard decision and
# the syndrome test), taken as 17.5.  A transcendental costs TRANS_SLOTS plain FP32
# issue slots (measured by paper_2407_11523_amd/calib/valu_rate: exp2 1.76, log2
# 1.74).  Peak issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 slots/s.
TRANS_SLOTS = 1.75
ALG_TRANS_PER_EDGE = 4.0
ALG_TRANS_PER_QUBIT = 3.0
ALG_OPS_PER_EDGE = 17.5


def algorithmic_slots(E, N):
    """FP32 issue slots of one iteration of one shot (E edges, N qubits)."""
    return TRANS_SLOTS * (ALG_TRANS_PER_EDGE * E + ALG_TRANS_PER_QUBIT * N) + ALG_OPS_PER_EDGE * E


# A second, finer count of the same work, itemised from the kernels' own evaluation
# (phi = 6 FP32 operations + one exp2 or log2; ln(1 + e^-|y|) = 3 operations + 2
# transcendentals):
#   check of degree d: 2d phi, d sign products, 2d - 1 leave-one-out sums, d sign
#                      applications, d clamps; syndrome test d + 1  -> 18d ops, 2d transcendentals
#   qubit of degree d with L labels present: d + 3 label sums, 9 posterior (EWAInit),
#                      5 hard decision, L lambdas (two softplus + 6 ops each), 2d
#                      output subtractions and clamps               -> 3d + 17 + 12L ops, 4L transcendentals
# so an iteration costs 21 E + 17 N + 12 sum(L) operations and 2 E + 4 sum(L)
# transcendentals; reported beside the algorithmic fraction.
def iteration_slots(code):
    """Itemised FP32 issue slots of one EWAInit iteration of one shot of `code`."""
    import numpy as np
    lab = code.labels()
    E = int((lab != 0).sum())
    N = code.n
    L = int(sum(len(set(int(x) for x in np.unique(lab[:, v])) - {0}) for v in range(N)))
    ops = 21 * E + 17 * N + 12 * L
    trans = 2 * E + 4 * L
    return ops + TRANS_SLOTS * trans


PEAK_SLOTS = 256 * 4 * 16 * 2.4e9
# two-sided normal quantile for a 95% family-wise interval over the 11 codes (0.05 / 11)
Z_FAMILY = 2.8376

# Large codes with HBM-resident messages: planar d=31 and toric L=32 at p = 0.10,
# 2^18 shots each, EWAInit-BP (chosen discount) with iter_max 200, structure-of-arrays kernel.
LARGE_CODES = list(configs.CONFIG5_CODES)
LARGE_P = configs.CONFIG5["p"]
LARGE_SHOTS = configs.CONFIG5["shots"]
LARGE_MAX_ITER = configs.CONFIG5["max_iter"]
LARGE_ALPHA = configs.alpha(5, "ewainit")
HBM_PEAK = 8.0e12   # bytes/s

# HBM traffic per launch from rocprofv3 counters (2 x FETCH_SIZE + WRITE_SIZE, the
# factors read off a 1 GiB device copy), valid only for the kernel sources they were
# taken on: a kernel whose sources hash differently reports traffic null.
KERNEL_SOURCES = {"decode_lds_kernel": ("bp4_decode.hip", "bp4_wide.h", "bp4_math.h", "bp4_internal.h"),
                  "decode_gather_kernel": ("bp4_gather.hip", "bp4_gather.h", "bp4_math.h", "bp4_internal.h",
                                           "bp4_walk.cpp")}
MEASURED_TRAFFIC = {"decode_lds_kernel": ("4fb5ef9c8464eddb", 3.910e+09),    # mixed batch, one launch
                    "decode_gather_kernel": ("4a8ae5b0af21aa50", 4.153e+12)}   # large codes, mean of 2 launches


def measured_traffic(kernel):
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2407_11523_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    sha, nbytes = MEASURED_TRAFFIC[kernel]
    return nbytes if h.hexdigest()[:16] == sha else None


def algorithmic_bytes(E, N):
    """Algorithmic HBM bytes of one EWAInit iteration of one shot with the state in HBM:
    the iteration state read and written once, every message (4 B per edge) and the
    posterior triple (12 B per qubit): 8 E + 24 N."""
    return 8 * E + 24 * N


def two_phase_bytes(E, N):
    """Bytes of a decoder that writes the check-to-qubit messages to HBM between its
    check and qubit phases: 16 E + 24 N (bounds its algorithmic fraction)."""
    return 16 * E + 24 * N


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=float, default=1.0, help="shot-count scale (1.0 = the named workload)")
    ap.add_argument("--no-plain", action="store_true", help="skip the per-code plain decoder")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--tuning-cache", default=None, help="autotuner cache file (default: the package's)")
    ap.add_argument("--no-tune", action="store_true", help="use the default lanes-per-shot pick")
    ap.add_argument("--no-large", action="store_true", help="skip the large-code (HBM kernels) measurement")
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP-graph replay of the step")
    ap.add_argument("--no-unrolled", action="store_true", help="skip the unrolled forward/adjoint measurement")
    ap.add_argument("--no-aewa", action="store_true", help="skip the AEWA-BP vs EWAInit-BP timing")
    ap.add_argument("--no-biased", action="store_true", help="skip the biased-noise XZZX curves")
    ap.add_argument("--no-serial", action="store_true", help="skip the serial-versus-flooding comparison")
    ap.add_argument("--no-qldpc", action="store_true", help="skip the bivariate bicycle and Chamon codes")
    ap.add_argument("--no-config2", action="store_true", help="skip the toric L=8 error-rate sweep")
    ap.add_argument("--only-large", action="store_true", help="run only the large-code (HBM kernels) measurement")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run 3 device-to-device copies of BYTES bytes (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(args.copy_calibration, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_calibration}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus_requested": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    import qecgen
    import paper_2407_11523_amd as P

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.only_large:
        print(json.dumps({"large_codes": run_large(torch, qecgen, P, dev)}), flush=True)
        return
    thr = qecgen.thresholds(P_ERR / 3, P_ERR / 3, P_ERR / 3)
    prm = P.Params(variant="ewainit", alpha=ALPHA, max_iter=MAX_ITER)
    items = []
    for i, (fam, size, mult) in enumerate(CODES):
        code = qecgen.make(fam, size)
        shots = max(1, int(round(BASE_SHOTS * mult * args.scale)))
        g = P.Graph(code.hx, code.hz, code.lx, code.lz, device=dev)
        pr = P.prior_llr(qecgen.depolarizing_probs(code.n, P_ERR), device=dev)
        err = torch.empty((shots, code.n), dtype=torch.uint8, device=dev)
        syn = torch.empty((shots, code.m), dtype=torch.uint8, device=dev)
        counts = torch.zeros(3, dtype=torch.int64, device=dev)
        items.append(dict(code=code, g=g, prior=pr, err=err, syn=syn, counts=counts, shots=shots,
                          slots=iteration_slots(code), seed=qecgen.config_seed(3, i, 0)))
    # launch shape per code from the autotuner (timed on up to 2^20 syndromes of each code)
    lanes = [0] * len(items)
    tuned = None
    if not args.no_tune:
        from paper_2407_11523_amd import tune
        for it in items:
            P.sample(it["g"], it["shots"], thr, it["seed"], err=it["err"], synd=it["syn"])
        kw = {"cache_path": args.tuning_cache} if args.tuning_cache else {}
        tuned = tune.tune_mixed([(it["g"], prm, it["prior"], it["syn"]) for it in items],
                                [tune.digest(it["code"].hx, it["code"].hz) for it in items],
                                [it["shots"] for it in items], **kw)
        lanes = tuned["lanes"]
        log(f"tuned lane mappings [group_lanes, block_shots] {lanes}, LDS budget {tuned['budget']} "
            f"({'cached' if tuned['cached'] else 'measured'} for {tuned['key']})")
    batch = P.MixedBatch([(it["g"], prm, it["prior"], it["syn"], G) for it, G in zip(items, lanes)])
    total_shots = sum(it["shots"] for it in items)
    log(f"workload: {len(items)} codes, {total_shots} shots per step")

    dec_ev = []

    def step(record):
        for it in items:
            P.sample(it["g"], it["shots"], thr, it["seed"], err=it["err"], synd=it["syn"])
        if record:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
        batch.run()
        if record:
            b.record()
            dec_ev.append((a, b))
        for it, o in zip(items, batch.outs):
            it["counts"].zero_()
            P.bookkeep(it["g"], it["err"], o["est"], counts=it["counts"])

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record()
    for _ in range(args.steps):
        step(True)
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1) / args.steps
    value = total_shots / (ms / 1e3)
    dec_ms = sum(a.elapsed_time(b) for a, b in dec_ev) / len(dec_ev)

    # work of the last step (every step decodes the same seeded syndromes)
    edge_updates = 0
    iters_total = 0
    slots = 0.0
    alg_slots = 0.0
    ler = {}
    fails = {}
    for it, o in zip(items, batch.outs):
        s = int(o["iters"].to(torch.int64).sum())
        iters_total += s
        edge_updates += s * it["code"].nnz
        slots += s * it["slots"]
        alg_slots += s * algorithmic_slots(it["code"].nnz, it["code"].n)
        c = it["counts"].cpu().numpy()
        fails[it["code"].name] = (int(c[1] + c[2]), it["shots"])
        ler[it["code"].name] = round(float(c[1] + c[2]) / it["shots"], 6)
    eups = edge_updates / (dec_ms / 1e3)
    achieved = alg_slots / (dec_ms / 1e3)
    achieved_itemised = slots / (dec_ms / 1e3)
    log(f"step {ms:.2f} ms, decode {dec_ms:.2f} ms, {eups:.3e} edge-updates/s, avg iters {iters_total / total_shots:.2f}")

    out = {
        "metric": "syndromes/s mixed-batch vs per-code plain BP, same GPU, LER in 95% CI",
        "value": value, "unit": "syndromes/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "mixed batch: planar d{5,7,9,11,13}, toric L{6,10,14}, XZZX L{5,9,13}, "
                               f"depolarizing p=0.08, 2^18 shots x 1:2:4 per size tier, EWAInit-BP alpha={ALPHA}, "
                               "iter_max 100, sample + one persistent decode launch + bookkeeping per step",
                   "shots_per_step": total_shots, "codes": len(items), "shot_scale": args.scale,
                   "lane_mapping": [list(x) if isinstance(x, (list, tuple)) else [int(x), 0] for x in lanes]},
        "decode_ms": dec_ms, "edge_updates_per_s": eups, "avg_iters": iters_total / total_shots,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12,
                     "unit": "T FP32 issue slots/s", "frac": achieved / PEAK_SLOTS,
                     "traffic": measured_traffic("decode_lds_kernel"),
                     "kernel": "decode_lds_kernel", "slots_per_edge_update": alg_slots / edge_updates,
                     "trans_slots": TRANS_SLOTS,
                     "itemised": {"slots_per_edge_update": slots / edge_updates,
                                  "achieved": achieved_itemised / 1e12, "frac": achieved_itemised / PEAK_SLOTS}},
        "ler": ler,
    }

    if not args.no_graph:
        # the same step recorded once as a HIP graph and replayed
        snap = [(o["est"].clone(), o["iters"].clone(), it["counts"].clone()) for it, o in zip(items, batch.outs)]
        cap = P.Captured(lambda: step(False))
        torch.cuda.synchronize()
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        g0.record()
        for _ in range(args.steps):
            cap.replay()
        g1.record()
        torch.cuda.synchronize()
        gms = g0.elapsed_time(g1) / args.steps
        same = all(torch.equal(a, o["est"]) and torch.equal(b, o["iters"]) and torch.equal(c, it["counts"])
                   for (a, b, c), it, o in zip(snap, items, batch.outs))
        out["graph"] = {"ms_per_step": gms, "value": total_shots / (gms / 1e3), "identical_to_eager": bool(same)}
        log(f"graph replay {gms:.2f} ms per step, identical outputs: {same}")
        del cap

    if not args.no_plain:
        plain_ms = 0.0
        same = True
        for it, o in zip(items, batch.outs):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record()
            r = P.decode_plain(it["g"], prm, it["prior"], it["syn"])
            b.record()
            torch.cuda.synchronize()
            plain_ms += a.elapsed_time(b)
            same = same and torch.equal(r["est"], o["est"]) and torch.equal(r["iters"], o["iters"])
            del r
            torch.cuda.empty_cache()
        out["plain_per_code"] = {"decode_ms": plain_ms, "value": total_shots / (plain_ms / 1e3),
                                 "unit": "syndromes/s", "speedup_of_mixed": plain_ms / dec_ms,
                                 "bit_identical": bool(same)}
        log(f"plain per-code decode {plain_ms:.1f} ms -> mixed is {plain_ms / dec_ms:.1f}x")

        # the mixed launch's own kernel run one code at a time (same lane mappings and
        # LDS budget): separates the batching gain from the kernel gain
        lds_ms = 0.0
        same = True
        for it, o, lane in zip(items, batch.outs, lanes):
            G, S = (lane if isinstance(lane, (list, tuple)) else (lane, 0))
            kw = dict(group_lanes=G, block_shots=S)
            if tuned is not None:
                kw["lds_bytes"] = tuned["budget"]
            P.decode(it["g"], prm, it["prior"], it["syn"][:4096], **kw)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record()
            r = P.decode(it["g"], prm, it["prior"], it["syn"], **kw)
            b.record()
            torch.cuda.synchronize()
            lds_ms += a.elapsed_time(b)
            same = same and torch.equal(r["est"], o["est"]) and torch.equal(r["iters"], o["iters"])
            del r
        out["lds_per_code"] = {"decode_ms": lds_ms, "value": total_shots / (lds_ms / 1e3), "unit": "syndromes/s",
                               "batching_gain": lds_ms / dec_ms, "kernel_gain": plain_ms / lds_ms,
                               "bit_identical": bool(same)}
        log(f"LDS kernel per code {lds_ms:.1f} ms: batching gain {lds_ms / dec_ms:.2f}x, "
            f"kernel gain over plain {plain_ms / lds_ms:.1f}x")

    if not args.no_cpu:
        from oracle import oracle as O
        O.build()
        threads = min(16, os.cpu_count() or 1)
        tot_shots = 0
        tot_t = 0.0
        tot_eu = 0
        in_ci = True
        ci = {}
        for it in items:
            code = it["code"]
            k = max(1, min(it["shots"], int(512 * it["shots"] / (BASE_SHOTS * args.scale))))
            e_o, s_o = O.sample(code.hx, code.hz, k, thr, seed=it["seed"], nthreads=threads)
            pi = O.prior_llr(qecgen.depolarizing_probs(code.n, P_ERR))
            t = time.perf_counter()
            ro = O.decode(code.hx, code.hz, O.Params(variant="ewainit", alpha=ALPHA, max_iter=MAX_ITER), pi, s_o,
                          nthreads=threads)
            tot_t += time.perf_counter() - t
            tot_shots += k
            tot_eu += int(ro["iters"].astype(np.int64).sum()) * int((code.labels() != 0).sum())
            _, co = O.bookkeep(code.hx, code.hz, code.lx, code.lz, e_o, ro["est"])
            # Wilson interval at family-wise 95% over the codes (Bonferroni: z for 0.05 / ncodes)
            lo, hi = O.wilson_ci(int(co[1] + co[2]), k, z=Z_FAMILY)
            nf, ns = fails[code.name]
            ok = lo <= nf / ns <= hi
            in_ci = in_ci and ok
            ci[code.name] = [round(lo, 5), round(hi, 5), ok]
        out["cpu_baseline"] = {"value": tot_shots / tot_t, "unit": "syndromes/s", "cores": threads, "kind": "oracle",
                               "sample": f"first 512 x (1|2|4) shots of each code ({tot_shots} shots), FP64 oracle, "
                                         f"OpenMP over shots"}
        model = ""
        try:
            with open("/proc/cpuinfo") as f:
                model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
        except OSError:
            pass
        out["oracle_host"] = {"cpu_model": model, "logical_cpus": os.cpu_count(), "threads": threads,
                              "us_per_shot": tot_t / tot_shots * 1e6, "edge_updates_per_s": tot_eu / tot_t}
        out["ler_in_oracle_ci"] = bool(in_ci)
        out["oracle_ci"] = ci
        log(f"oracle {tot_shots / tot_t:.0f} shots/s on {threads} threads")

    if not args.no_unrolled:
        out["unrolled"] = run_unrolled(torch, qecgen, P, dev)

    if not args.no_config2:
        out["toric_sweep"] = run_config2(torch, qecgen, P, dev)
    if not args.no_aewa:
        out["aewa"] = run_aewa(torch, qecgen, P, dev)
    if not args.no_biased:
        out["biased_xzzx"] = run_biased(torch, qecgen, P, dev)
    if not args.no_serial:
        out["serial"] = run_serial(torch, qecgen, P, dev)
    if not args.no_qldpc:
        out["other_qldpc"] = run_qldpc(torch, qecgen, P, dev)

    if not args.no_large:
        del batch, items
        torch.cuda.empty_cache()
        out["large_codes"] = run_large(torch, qecgen, P, dev)

    out["wall_s"] = wall
    print(json.dumps(out), flush=True)


def wilson_ci(k, n, z=1.959963984540054):
    """Wilson score interval of a binomial proportion k / n."""
    if n == 0:
        return (0.0, 1.0)
    ph = k / n
    den = 1 + z * z / n
    ctr = (ph + z * z / (2 * n)) / den
    half = z * (ph * (1 - ph) / n + z * z / (4 * n * n)) ** 0.5 / den
    return (max(0.0, ctr - half), min(1.0, ctr + half))


def _crossing(ps, a, b):
    """Error rate where curve b - a changes sign (linear interpolation), or None."""
    for j in range(len(ps) - 1):
        d0, d1 = b[j] - a[j], b[j + 1] - a[j + 1]
        if d0 < 0 <= d1 or d0 <= 0 < d1:
            return ps[j] + (ps[j + 1] - ps[j]) * (-d0) / (d1 - d0)
    return None


def run_config2(torch, qecgen, P, dev):
    """Toric L=8 sweep of section IV-B: p = 0.02 .. 0.16 in 8 steps, 2^20 shots per point,
    Momentum-BP (gamma 0), AdaGrad-BP (alpha 5) and EWAInit-BP with the chosen discounts,
    iter_max 100: decode throughput, edge updates/s, iterations and LER with its Wilson
    95% interval per point.  EWAInit also on toric L=4 and 6 for the curves' crossing
    (the paper reads about 13.6% for L = 4, 6, 8 under parallel scheduling)."""
    c2 = configs.CONFIG2
    shots = c2["shots"]
    ps = list(c2["p"])
    rows = []
    curves = {}
    for L in (8, 6, 4):
        code = qecgen.toric(L)
        g = P.Graph(code.hx, code.hz, code.lx, code.lz, device=dev)
        variants = ("momentum", "adagrad", "ewainit") if L == 8 else ("ewainit",)
        for variant in variants:
            alpha = configs.alpha(2, variant)
            prm = P.Params(variant=variant, alpha=alpha, gamma=configs.MOMENTUM_GAMMA, max_iter=c2["max_iter"])
            lers = []
            for j, p in enumerate(ps):
                seed = qecgen.config_seed(2, 0, j) if L == 8 else qecgen.config_seed(2, L, j)
                err, syn = P.sample(g, shots, qecgen.thresholds(p / 3, p / 3, p / 3), seed=seed)
                pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p), device=dev)
                P.decode(g, prm, pr, syn[:4096])
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                r = P.decode(g, prm, pr, syn)
                b.record()
                _, cnt = P.bookkeep(g, err, r["est"])
                torch.cuda.synchronize()
                ms = a.elapsed_time(b)
                it_sum = int(r["iters"].to(torch.int64).sum())
                fails = int(cnt[1] + cnt[2])
                lo, hi = wilson_ci(fails, shots)
                lers.append(fails / shots)
                rows.append({"L": L, "variant": variant, "alpha": alpha, "p": p, "decode_ms": ms,
                             "syndromes_per_s": shots / (ms / 1e3), "edge_updates_per_s": it_sum * g.nnz / (ms / 1e3),
                             "avg_iters": it_sum / shots, "converged": float(r["conv"].float().mean()),
                             "ler": fails / shots, "ler_ci95": [lo, hi]})
                del r, err, syn
            curves[(L, variant)] = lers
    cross = {f"L{a}_L8": _crossing(ps, curves[(a, "ewainit")], curves[(8, "ewainit")]) for a in (4, 6)}
    l8 = [r for r in rows if r["L"] == 8]
    tot_ms = sum(r["decode_ms"] for r in l8)
    log("config2 toric L=8: " + ", ".join(f"{r['variant'][:3]} p{r['p']}: {r['syndromes_per_s'] / 1e6:.0f}M/s "
                                           f"LER {r['ler']:.4f}" for r in l8 if r["p"] in (0.02, 0.08, 0.16)))
    log(f"config2 EWAInit crossings {cross} (paper: about 0.136)")
    return {"workload": "toric L=8, depolarizing p = 0.02..0.16 (8 points), 2^20 shots per point, Momentum-BP "
                        f"(alpha {configs.alpha(2, 'momentum')}, gamma 0), AdaGrad-BP (alpha 5), EWAInit-BP "
                        f"(alpha {configs.alpha(2, 'ewainit')}), iter_max 100; EWAInit also on toric L=4, 6",
            "rows": rows, "syndromes_per_s_l8": len(l8) * shots / (tot_ms / 1e3),
            "ewainit_crossing": cross, "paper_crossing": 0.136}


# Table II of the paper (runtime per decode on planar codes, hardware not stated):
# EWAInit-BP and AEWA-BP in ms at physical error rates 1e-2, 6e-2, 1e-1, 2e-1.
PAPER_TABLE2 = {0.01: (1.1, 1.6), 0.06: (3.7, 27.9), 0.10: (7.7, 81.9), 0.20: (20.1, 240.6)}


def run_aewa(torch, qecgen, P, dev):
    """EWAInit-BP (alpha 0.5) and AEWA-BP (11 discounts 1 .. 0) on planar d=3, 7, 11, 2^16
    shots each, iter_max 100, at the physical error rates of the paper's Table II."""
    shots = 1 << 16
    res = {"workload": "planar d=3, 7, 11, 2^16 shots each, iter_max 100, EWAInit alpha 0.5 vs AEWA 11 discounts "
                       "from 1 to 0, at the error rates of the paper's Table II",
           "rows": []}
    for p in sorted(PAPER_TABLE2):
        thr = qecgen.thresholds(p / 3, p / 3, p / 3)
        row = {"p": p, "paper_ms": {"ewainit": PAPER_TABLE2[p][0], "aewa": PAPER_TABLE2[p][1]}}
        tot = {"ewainit": 0.0, "aewa": 0.0}
        tot_it = {"ewainit": 0, "aewa": 0}
        for i, d in enumerate((3, 7, 11)):
            code = qecgen.planar(d)
            g = P.Graph(code.hx, code.hz, code.lx, code.lz, device=dev)
            pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p), device=dev)
            err, syn = P.sample(g, shots, thr, seed=qecgen.config_seed(6, i, int(p * 100)))
            for name, prm in (("ewainit", P.Params(variant="ewainit", alpha=ALPHA_EXTRA, max_iter=100)),
                              ("aewa", P.Params(variant="aewa", alpha=1.0, alpha_last=0.0, alpha_steps=11,
                                                max_iter=100))):
                P.decode(g, prm, pr, syn[:1024])
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                r = P.decode(g, prm, pr, syn)
                b.record()
                torch.cuda.synchronize()
                ms = a.elapsed_time(b)
                _, cnt = P.bookkeep(g, err, r["est"])
                tot[name] += ms
                tot_it[name] += int(r["iters"].to(torch.int64).sum())
                row[f"d{d}_{name}"] = {"ms": ms, "syndromes_per_s": shots / (ms / 1e3),
                                        "ler": float(cnt[1] + cnt[2]) / shots,
                                        "avg_iters": float(r["iters"].float().mean()),
                                        "max_iters": int(r["iters"].max())}
        row["aewa_over_ewainit_time"] = tot["aewa"] / tot["ewainit"]
        # the work ratio (a sequential decoder's time ratio): iterations summed over all shots
        row["aewa_over_ewainit_iterations"] = tot_it["aewa"] / tot_it["ewainit"]
        row["paper_aewa_over_ewainit_time"] = PAPER_TABLE2[p][1] / PAPER_TABLE2[p][0]
        res["rows"].append(row)
        log(f"aewa p={p}: AEWA/EWAInit time {row['aewa_over_ewainit_time']:.1f}, iterations "
            f"{row['aewa_over_ewainit_iterations']:.1f} (paper time {row['paper_aewa_over_ewainit_time']:.1f}); "
            f"max iterations per shot d3/d7/d11 {[row[f'd{d}_aewa']['max_iters'] for d in (3, 7, 11)]}")
    return res


def run_serial(torch, qecgen, P, dev):
    """Serial (Algorithm 1) against flooding (Algorithm 2) EWAInit (the toric sweep's discount), iter_max 100, on
    toric L=4, 6, 8 with 2^16 shots at p = 0.06 ... 0.16: LER, iterations and throughput (the
    paper reads the serial crossing at about 15%, the flooding one at about 13.6%)."""
    shots = 1 << 16
    ps = (0.06, 0.10, 0.14, 0.16)
    rows = []
    for i, L in enumerate((4, 6, 8)):
        code = qecgen.toric(L)
        g = P.Graph(code.hx, code.hz, code.lx, code.lz, device=dev)
        for j, p in enumerate(ps):
            pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p), device=dev)
            err, syn = P.sample(g, shots, qecgen.thresholds(p / 3, p / 3, p / 3), seed=qecgen.config_seed(8, i, j))
            row = {"L": L, "p": p}
            for name, serial in (("flooding", False), ("serial", True)):
                prm = P.Params(variant="ewainit", alpha=configs.alpha(2, "ewainit"), max_iter=100, serial=serial)
                P.decode(g, prm, pr, syn[:512])
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                r = P.decode(g, prm, pr, syn)
                b.record()
                torch.cuda.synchronize()
                _, cnt = P.bookkeep(g, err, r["est"])
                row[name] = {"ler": float(cnt[1] + cnt[2]) / shots, "avg_iters": float(r["iters"].float().mean()),
                             "syndromes_per_s": shots / (a.elapsed_time(b) / 1e3)}
            rows.append(row)
    log("serial vs flooding: " + ", ".join(f"L{r['L']} p{r['p']}: {r['serial']['ler']:.4f}/{r['flooding']['ler']:.4f}"
                                            for r in rows if r["p"] == 0.14))
    return {"workload": f"toric L=4, 6, 8, 2^16 shots, EWAInit alpha {configs.alpha(2, 'ewainit')}, iter_max 100, "
                        "serial vs flooding",
            "rows": rows}


def run_biased(torch, qecgen, P, dev):
    """XZZX L=5, 7, 9 under biased noise (p_Z = 2p/3, p_X = p_Y = p/6), iter_max 100, 2^16
    shots per point: the LER curves of EWAInit at alpha 0.5 and where the L=5 and L=9 curves
    cross (the paper reads about 10% for EWAInit under parallel scheduling), then the same
    crossings (L5/L9 and L7/L9) for every discount of the paper's grid 0, 0.1, ..., 1 on the
    same syndromes (alpha 1 is traditional BP)."""
    shots = 1 << 16
    ps = (0.04, 0.06, 0.08, 0.10, 0.12, 0.14, 0.16, 0.18, 0.20, 0.22)
    sizes = (5, 7, 9)
    cases = {}
    for i, L in enumerate(sizes):
        code = qecgen.xzzx(L)
        g = P.Graph(code.hx, code.hz, code.lx, code.lz, device=dev)
        cases[L] = []
        for j, p in enumerate(ps):
            probs = qecgen.biased_probs(code.n, p)
            err, syn = P.sample(g, shots, qecgen.thresholds(*probs[0]), seed=qecgen.config_seed(7, i, j))
            cases[L].append((g, err, syn, P.prior_llr(probs, device=dev)))

    def curves(alpha):
        prm = P.Params(variant="ewainit", alpha=alpha, max_iter=100)
        ler = {}
        for L in sizes:
            ler[L] = []
            for g, err, syn, pr in cases[L]:
                r = P.decode(g, prm, pr, syn)
                _, cnt = P.bookkeep(g, err, r["est"])
                ler[L].append(float(cnt[1] + cnt[2]) / shots)
        return ler

    def cross(a, b):   # first sign change of b - a, linearly interpolated
        for j in range(len(ps) - 1):
            d0, d1 = b[j] - a[j], b[j + 1] - a[j + 1]
            if d0 < 0 <= d1 or d0 <= 0 < d1:
                return ps[j] + (ps[j + 1] - ps[j]) * (-d0) / (d1 - d0)
        return None

    ler = curves(ALPHA_EXTRA)
    x59 = cross(ler[5], ler[9])
    log(f"biased XZZX: L=5/9 LER curves cross near p = {x59}")
    sweep = []
    for k in range(11):
        lk = ler if k == round(ALPHA_EXTRA * 10) else curves(k / 10)
        sweep.append({"alpha": k / 10, "crossing_L5_L9": cross(lk[5], lk[9]), "crossing_L7_L9": cross(lk[7], lk[9]),
                      "ler_L9": lk[9]})
    log("biased XZZX crossings L5/L9 by alpha: " +
        ", ".join(f"{r['alpha']:.1f}: {r['crossing_L5_L9']}" for r in sweep))
    return {"workload": "XZZX L=5, 7, 9, p_Z = 2p/3, p_X = p_Y = p/6, EWAInit, iter_max 100, 2^16 shots per point",
            "p": list(ps), "alpha": ALPHA_EXTRA, "ler": {f"L{L}": v for L, v in ler.items()}, "crossing_L5_L9": x59,
            "paper_crossing": 0.10, "alpha_sweep": sweep}


def run_qldpc(torch, qecgen, P, dev):
    """Other qLDPC codes (section IV-C): bivariate bicycle codes [[72,12,6]], [[90,8,10]],
    [[108,8,10]], [[144,12,12]] and 3D Chamon codes d = 3, 4 (degree-6 checks and qubits,
    the wide flooding LDS kernel) under depolarizing noise: LER of EWAInit-BP (alpha 0.5)
    and traditional BP, iter_max 100, 2^16 shots per point, and decode throughput."""
    shots = 1 << 16
    ps = (0.02, 0.04, 0.06, 0.08)
    codes = [("bb", 72), ("bb", 90), ("bb", 108), ("bb", 144), ("chamon", 3), ("chamon", 4)]
    rows = []
    for i, (fam, size) in enumerate(codes):
        code = qecgen.make(fam, size)
        g = P.Graph(code.hx, code.hz, code.lx, code.lz, device=dev)
        row = {"code": code.name, "n": code.n, "k": code.k, "p": list(ps)}
        for variant, alpha in (("ewainit", ALPHA_EXTRA), ("bp", 1.0), ("aewa", 1.0)):
            prm = P.Params(variant=variant, alpha=alpha, max_iter=100,
                           **(dict(alpha_last=0.0, alpha_steps=11) if variant == "aewa" else {}))
            lers, rates = [], []
            for j, p in enumerate(ps):
                err, syn = P.sample(g, shots, qecgen.thresholds(p / 3, p / 3, p / 3),
                                    seed=qecgen.config_seed(9, i, j))
                pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p), device=dev)
                P.decode(g, prm, pr, syn)                       # warm-up
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                r = P.decode(g, prm, pr, syn)
                b.record()
                _, cnt = P.bookkeep(g, err, r["est"])
                torch.cuda.synchronize()
                lers.append(float(cnt[1] + cnt[2]) / shots)
                rates.append(shots / (a.elapsed_time(b) / 1e3))
            row[variant] = {"ler": lers, "syndromes_per_s": rates}
        # the paper states no discount for these codes: EWAInit over alpha at p = 0.04
        sweep = {}
        err, syn = P.sample(g, shots, qecgen.thresholds(0.04 / 3, 0.04 / 3, 0.04 / 3), seed=qecgen.config_seed(9, i, 9))
        pr = P.prior_llr(qecgen.depolarizing_probs(code.n, 0.04), device=dev)
        for alpha in (0.5, 0.6, 0.7, 0.8, 0.9, 1.0):
            r = P.decode(g, P.Params(variant="ewainit", alpha=alpha, max_iter=100), pr, syn)
            _, cnt = P.bookkeep(g, err, r["est"])
            torch.cuda.synchronize()
            sweep[str(alpha)] = float(cnt[1] + cnt[2]) / shots
        row["ewainit_alpha_sweep_p0.04"] = sweep
        rows.append(row)
        log(f"{code.name}: LER EWAInit {[round(x, 4) for x in row['ewainit']['ler']]} "
            f"BP {[round(x, 4) for x in row['bp']['ler']]} AEWA {[round(x, 4) for x in row['aewa']['ler']]} "
            f"alpha sweep p=0.04 {sweep}")
    return {"workload": "bivariate bicycle n = 72, 90, 108, 144 and 3D Chamon d = 3, 4, depolarizing p = 0.02-0.08, "
                        "2^16 shots per point, EWAInit-BP alpha 0.5, BP and AEWA-BP (11 discounts 1 to 0), "
                        "iter_max 100; EWAInit over alpha at p = 0.04",
            "rows": rows}


def run_unrolled(torch, qecgen, P, dev):
    """Unrolled EWAInit forward + adjoint: planar d=9, p=0.06, 65,536 shots, T=32, checkpoints every 8."""
    code = qecgen.planar(9)
    T, K, shots, p = 32, 8, 1 << 16, 0.06
    g = P.Graph(code.hx, code.hz, code.lx, code.lz, device=dev)
    err, syn = P.sample(g, shots, qecgen.thresholds(p / 3, p / 3, p / 3), seed=qecgen.config_seed(4, 0, 0))
    alpha = torch.full((T,), ALPHA_EXTRA, dtype=torch.float32, device=dev, requires_grad=True)
    prior = P.prior_llr(qecgen.depolarizing_probs(code.n, p), device=dev).clone().requires_grad_(True)
    times = []
    for rep in range(3):
        alpha.grad = None
        prior.grad = None
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        c = torch.cuda.Event(enable_timing=True)
        a.record()
        loss = P.unrolled_loss(g, alpha, prior, syn, err, T, K)
        b.record()
        loss.backward()
        c.record()
        torch.cuda.synchronize()
        times.append((a.elapsed_time(b), b.elapsed_time(c)))
    fwd, bwd = min(times, key=lambda x: x[0] + x[1])
    eu = shots * T * g.nnz
    log(f"unrolled: forward {fwd:.2f} ms, backward {bwd:.2f} ms")
    res = {"workload": "planar d=9, p=0.06, 65,536 shots, T=32 unrolled EWAInit iterations, checkpoints every 8, "
                       "loss and gradients w.r.t. alpha_t and the priors",
           "forward_ms": fwd, "backward_ms": bwd, "loss": float(loss.detach()),
           "shots_per_s_forward_backward": shots / ((fwd + bwd) / 1e3),
           "edge_updates_per_s_forward": eu / (fwd / 1e3),
           # the forward's state (messages and Q) read and written once per shot-iteration
           "forward_algorithmic_bytes_per_shot_iteration": algorithmic_bytes(g.nnz, g.n),
           "forward_algorithmic_gb_s": shots * T * algorithmic_bytes(g.nnz, g.n) / (fwd / 1e3) / 1e9,
           "forward_hbm_frac": shots * T * algorithmic_bytes(g.nnz, g.n) / (fwd / 1e3) / 8e12,
           "grad_alpha_norm": float(alpha.grad.norm()), "grad_prior_norm": float(prior.grad.norm())}
    # the same batch unrolled as Momentum-BP: a step and a decay per iteration (starting
    # from the toric sweep's step and gamma 0)
    params = torch.tensor([[MOMENTUM_ALPHA, 0.0]] * T, dtype=torch.float32, device=dev, requires_grad=True)
    times = []
    for rep in range(3):
        params.grad = None
        prior.grad = None
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        c = torch.cuda.Event(enable_timing=True)
        a.record()
        loss_m = P.unrolled_loss(g, params, prior, syn, err, T, K, variant="momentum")
        b.record()
        loss_m.backward()
        c.record()
        torch.cuda.synchronize()
        times.append((a.elapsed_time(b), b.elapsed_time(c)))
    fwd_m, bwd_m = min(times, key=lambda x: x[0] + x[1])
    log(f"unrolled momentum: forward {fwd_m:.2f} ms, backward {bwd_m:.2f} ms")
    mom_bytes = 8 * g.nnz + 72 * g.n   # messages, Q, g and M read and written once per shot-iteration
    res["momentum"] = {"workload": "the same batch, T=32 unrolled Momentum-BP iterations, loss and gradients w.r.t. "
                                   "the steps alpha_t, the decays gamma_t and the priors",
                       "forward_ms": fwd_m, "backward_ms": bwd_m, "loss": float(loss_m.detach()),
                       "forward_algorithmic_bytes_per_shot_iteration": mom_bytes,
                       "forward_hbm_frac": shots * T * mom_bytes / (fwd_m / 1e3) / 8e12,
                       "grad_params_norm": float(params.grad.norm()), "grad_prior_norm": float(prior.grad.norm())}
    return res


def run_large(torch, qecgen, P, dev):
    """Decode 2^18 shots of each large code with the single-pass HBM kernel (the automatic
    choice) and, on the same syndromes, with the two-phase SOA kernel; HBM roofline of
    the single-pass kernel."""
    thr = qecgen.thresholds(LARGE_P / 3, LARGE_P / 3, LARGE_P / 3)
    prm = P.Params(variant="ewainit", alpha=LARGE_ALPHA, max_iter=LARGE_MAX_ITER)
    warm = P.Params(variant="ewainit", alpha=LARGE_ALPHA, max_iter=2)
    res = {"workload": f"planar d=31 and toric L=32, depolarizing p=0.10, 2^18 shots each, EWAInit-BP "
                       f"alpha={LARGE_ALPHA}, iter_max 200, messages in HBM (single-pass kernel; the two-phase "
                       f"structure-of-arrays kernel timed on the same syndromes)",
           "codes": {}}
    tot = {"gather": 0.0, "soa": 0.0}
    tot_bytes = tot_shots = tot_eu = 0.0
    for i, (fam, size) in enumerate(LARGE_CODES):
        code = qecgen.make(fam, size)
        # the lattice positions order the single-pass kernel's walk (strips of the layout)
        g = P.Graph(code.hx, code.hz, code.lx, code.lz, device=dev, coords=code.coords)
        pr = P.prior_llr(qecgen.depolarizing_probs(code.n, LARGE_P), device=dev)
        err, syn = P.sample(g, LARGE_SHOTS, thr, seed=qecgen.config_seed(5, i, 0))
        row = {}
        results = {}
        for kernel in ("gather", "soa"):
            nbytes_ws = (g.gather_workspace_bytes(prm, LARGE_SHOTS) if kernel == "gather"
                         else g.soa_workspace_bytes(prm, LARGE_SHOTS))
            ws = torch.empty(nbytes_ws, dtype=torch.uint8, device=dev)
            P.decode(g, warm, pr, syn[:256], kernel=kernel, ws=ws)          # warm-up (loads the code object)
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            r = P.decode(g, prm, pr, syn, kernel=kernel, ws=ws)
            b.record()
            torch.cuda.synchronize()
            row[kernel + "_ms"] = a.elapsed_time(b)
            results[kernel] = r
            del ws
            torch.cuda.empty_cache()
        r = results["gather"]
        same = all(torch.equal(r[k], results["soa"][k]) for k in ("est", "conv", "iters"))
        ms = row["gather_ms"]
        _, counts = P.bookkeep(g, err, r["est"])
        it_sum = int(r["iters"].to(torch.int64).sum())
        nbytes = it_sum * algorithmic_bytes(g.nnz, g.n)
        c = counts.cpu().numpy()
        res["codes"][code.name] = {
            "decode_ms": ms, "soa_decode_ms": row["soa_ms"], "speedup_vs_soa": row["soa_ms"] / ms,
            "bitwise_equal_to_soa": same,
            "syndromes_per_s": LARGE_SHOTS / (ms / 1e3),
            "edge_updates_per_s": it_sum * g.nnz / (ms / 1e3), "avg_iters": it_sum / LARGE_SHOTS,
            "converged": float(r["conv"].float().mean()), "ler": float(c[1] + c[2]) / LARGE_SHOTS,
            "algorithmic_gb_s": nbytes / (ms / 1e3) / 1e9,
            "soa_algorithmic_gb_s": nbytes / (row["soa_ms"] / 1e3) / 1e9,
            "algorithmic_bytes_per_shot_iteration": algorithmic_bytes(g.nnz, g.n),
            "algorithmic_bytes_per_launch": nbytes,
            "soa_two_phase_cap": algorithmic_bytes(g.nnz, g.n) / two_phase_bytes(g.nnz, g.n)}
        log(f"{code.name}: single-pass {ms:.1f} ms ({nbytes / (ms / 1e3) / 1e9:.0f} GB/s algorithmic), "
            f"two-phase SOA {row['soa_ms']:.1f} ms, bitwise equal {same}")
        for k in tot:
            tot[k] += row[k + "_ms"]
        tot_bytes += nbytes
        tot_shots += LARGE_SHOTS
        tot_eu += it_sum * g.nnz
        del r, results, err, syn
        torch.cuda.empty_cache()
    launches = len(LARGE_CODES)   # one persistent launch per code
    achieved = tot_bytes / (tot["gather"] / 1e3)
    res["syndromes_per_s"] = tot_shots / (tot["gather"] / 1e3)
    res["edge_updates_per_s"] = tot_eu / (tot["gather"] / 1e3)
    res["soa_syndromes_per_s"] = tot_shots / (tot["soa"] / 1e3)
    res["roofline"] = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK, "traffic": measured_traffic("decode_gather_kernel"),
                       "kernel": "decode_gather_kernel", "launches": launches,
                       "algorithmic_bytes_per_launch": tot_bytes / launches,
                       "soa_frac": tot_bytes / (tot["soa"] / 1e3) / HBM_PEAK}
    return res

if __name__ == "__main__":
    main()
