"""GPU: bp4_decode_mixed_noalloc (queue heads in the library's static device array)
against bp4_decode_mixed (queue heads in a caller workspace), through the C ABI.

Both run the same kernel, so their outputs must be bit-identical: two calls in a
row, the second with fewer codes and fewer shots, so the second call starts from
the heads the first one left behind and must clear them itself."""
import ctypes
import sys

import numpy as np
import pytest

import qecgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2407_11523_amd as P  # noqa: E402
from paper_2407_11523_amd import _lib  # noqa: E402
from paper_2407_11523_amd import api as A  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_batch(spec, p=0.08, seed0=900):
    entries = []
    for i, (fam, size, shots, variant, alpha) in enumerate(spec):
        code = qecgen.make(fam, size)
        g = P.Graph(code.hx, code.hz, code.lx, code.lz)
        _, syn = P.sample(g, shots, qecgen.thresholds(p / 3, p / 3, p / 3), seed=seed0 + i)
        pr = P.prior_llr(qecgen.depolarizing_probs(code.n, p))
        entries.append((g, P.Params(variant=variant, alpha=alpha, max_iter=100), pr, syn, 0))
    return entries


def run_noalloc(entries):
    """The batch through bp4_decode_mixed_noalloc; outputs allocated here, by the caller."""
    outs = []
    arr = (_lib.CodeBatch * len(entries))()
    for i, (g, prm, prior, synd, _) in enumerate(entries):
        shots = synd.shape[0]
        o = {"est": torch.full((shots, g.n), 0xEE, dtype=torch.uint8, device="cuda"),
             "conv": torch.full((shots,), 0xEE, dtype=torch.uint8, device="cuda"),
             "iters": torch.full((shots,), -1, dtype=torch.int32, device="cuda")}
        outs.append(o)
        arr[i] = _lib.CodeBatch(g.handle.value, g.dev.data_ptr(), prm.c(), shots, prior.data_ptr(), synd.data_ptr(),
                                o["est"].data_ptr(), o["conv"].data_ptr(), o["iters"].data_ptr(), 0, 0)
    lib = _lib.load()
    _lib.check(lib.bp4_decode_mixed_noalloc(len(entries), arr, A._stream(torch.device("cuda"))))
    torch.cuda.synchronize()
    return outs


def test_noalloc_equals_workspace_entry_twice():
    first = [("planar", 7, 6000, "ewainit", 0.6), ("toric", 10, 4000, "momentum", 0.9),
             ("xzzx", 9, 5000, "adagrad", 5.0), ("planar", 5, 3000, "bp", 1.0)]
    second = [("toric", 6, 1500, "ewainit", 0.6), ("planar", 9, 900, "ewainit", 0.6)]
    for spec in (first, second):
        entries = make_batch(spec)
        ref = P.decode_mixed(entries)
        torch.cuda.synchronize()
        got = run_noalloc(entries)
        for (fam, size, shots, variant, _), r, o in zip(spec, ref, got):
            say("noalloc", fam, size, shots, variant, float(o["iters"].float().mean()))
            for k in ("est", "conv", "iters"):
                assert torch.equal(r[k], o[k]), (fam, size, k)


def test_noalloc_rejects_sizes_beyond_its_array():
    lib = _lib.load()
    arr = (_lib.CodeBatch * 17)()
    assert lib.bp4_decode_mixed_noalloc(17, arr, None) == -1
    assert lib.bp4_decode_mixed_noalloc(0, arr, None) == -1
    assert b"16" in lib.bp4_last_error()
