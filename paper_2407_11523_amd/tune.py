"""Autotuner of the LDS decode kernel's launch shape.

For each code it times the feasible lane mappings on a sample of the code's own
syndromes: wave groups of G = 4 ... 64 lanes per shot, and block slots of S
shots sharing a 512-lane workgroup (the S values of best lane use that fit).  In a mixed launch every workgroup reserves
the largest LDS layout of the batch, which sets the occupancy of all codes, so
the tuner times each code under each candidate LDS budget (the single-code
launch reserves that budget too) and keeps the budget whose summed, shot-scaled
time is smallest.  Choices are cached per device in tuning_cache.json.
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os
from typing import Dict, List, Optional, Sequence

import torch

from ._lib import check, load
from .api import Graph, Params, decode

PKG = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(PKG, "tuning_cache.json")
GROUP_SIZES = (4, 8, 16, 32, 64)
BLOCK = 512
MAX_BLOCK_CANDS = 4
# LDS per 512-lane workgroup that leaves 4, 3 and 2 workgroups per CU: 160 KiB / k
# rounded down to 2 KiB, since LDS is allocated in granules (budgets of 54,613 and
# 54,272 bytes held only two workgroups; layouts up to 51,452 bytes held three)
BUDGETS = (40960, 53248, 81920)


def layout_bytes(g: Graph, params: Params, lanes: int, block_shots: int = 0) -> Optional[int]:
    b = ctypes.c_size_t()
    cp = params.c()
    rc = load().bp4_lds_layout_bytes(g.handle, ctypes.byref(cp), int(lanes), int(block_shots), ctypes.byref(b))
    return int(b.value) if rc == 0 else None


def lane_use(m: int, n: int, G: int, S: int) -> float:
    """Share of issued (lane, item) pairs that carry a check or a qubit."""
    def use(k):
        if S:
            return S * k / (BLOCK * -(-S * k // BLOCK))
        return k / (G * -(-k // G))
    return 0.5 * (use(m) + use(n))


def candidates(g: Graph, params: Params, budget: int) -> List[tuple]:
    """(G, S) mappings whose layout fits `budget`: every wave group size and the
    block-slot counts of best lane use (ties: fewer slots)."""
    out = [(G, 0) for G in GROUP_SIZES if (layout_bytes(g, params, G) or budget + 1) <= budget]
    blocks = []
    for S in range(1, BLOCK + 1):
        lb = layout_bytes(g, params, 0, S)
        if lb is None or lb > budget:
            break
        blocks.append((-lane_use(g.m, g.n, 0, S), S))
    blocks.sort()
    out += [(0, S) for _, S in blocks[:MAX_BLOCK_CANDS]]
    return out


def code_key(g: Graph, params: Params, hx_hz_digest: str) -> str:
    return f"{g.m}x{g.n}:{g.nnz}:{hx_hz_digest}:{params.variant}:{params.max_iter}"


def digest(hx, hz) -> str:
    h = hashlib.sha1()
    h.update(bytes(memoryview(hx.tobytes())))
    h.update(bytes(memoryview(hz.tobytes())))
    return h.hexdigest()[:16]


def device_key(device=None) -> str:
    # the ISA and the CU count set the launch shapes; the marketing name varies by driver
    p = torch.cuda.get_device_properties(device)
    arch = getattr(p, "gcnArchName", "").split(":")[0]
    return f"{arch}:{p.multi_processor_count}cu"


def _time(fn, reps: int = 3) -> float:
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def _load_cache(path: str) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _save_cache(c: dict, path: str) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_mixed(entries: Sequence, digests: Sequence[str], shots_total: Sequence[int],
               sample: int = 1 << 20, use_cache: bool = True, save: bool = True,
               cache_path: str = CACHE) -> Dict:
    """Pick the lane mapping of every code of a mixed batch.

    entries: (graph, params, prior, synd) per code; synd holds at least `sample`
    rows (fewer are used as they are).  shots_total: shots per code in the real
    run (weights of the per-code times).  Returns {"lanes": [[G, S], ...],
    "budget": B, "table": ...}."""
    dev = entries[0][0].dev.device
    keys = [code_key(g, p, d) for (g, p, _, _), d in zip(entries, digests)]
    batch_key = device_key(dev) + ":slots512|" + "|".join(keys)
    cache = _load_cache(cache_path) if use_cache else {}
    if batch_key in cache:
        return dict(cache[batch_key], cached=True, key=batch_key.split("|")[0])
    table = {}
    best = None
    for B in BUDGETS:
        total = 0.0
        lanes = []
        rows = []
        for (g, p, prior, synd), k, S in zip(entries, keys, shots_total):
            s = synd[:min(sample, synd.shape[0])]
            cands = []
            for G, BS in candidates(g, p, B):
                ms = _time(lambda: decode(g, p, prior, s, group_lanes=G, block_shots=BS, lds_bytes=B))
                cands.append((ms, G, BS))
            if not cands:
                total = float("inf")
                lanes.append([0, 0])
                continue
            ms, G, BS = min(cands)
            lanes.append([G, BS])
            total += ms * S / max(1, s.shape[0])
            rows.append({"code": k, "G": G, "S": BS, "ms": ms,
                         "cands": {f"{g_}x{s_}": t for t, g_, s_ in cands}})
        table[str(B)] = {"predicted_ms": total, "codes": rows}
        if best is None or total < best[0]:
            best = (total, B, lanes)
    res = {"lanes": best[2], "budget": best[1], "predicted_ms": best[0], "table": table}
    if save:
        cache[batch_key] = res
        _save_cache(cache, cache_path)
    return dict(res, cached=False, key=batch_key.split("|")[0])
