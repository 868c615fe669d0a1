"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, builds graphs, and rejects bad arguments before launching anything."""
import ctypes
import os
import re

import numpy as np
import pytest

import qecgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bp4.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2407_11523_amd import _lib
    return _lib.load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bp4_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol(lib):
    from paper_2407_11523_amd import _lib
    names = declared_functions()
    assert "bp4_decode" in names and "bp4_sample" in names
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, name


def _graph(code, flags=0):
    from paper_2407_11523_amd import Graph
    return Graph(code.hx, code.hz, code.lx, code.lz, upload=False,
                 allow_anticommuting=bool(flags))


@pytest.mark.parametrize("make", [lambda: qecgen.planar(3), lambda: qecgen.toric(8), lambda: qecgen.xzzx(5),
                                  lambda: qecgen.planar(31)])
def test_graph_info_and_canonical_edges(lib, make):
    code = make()
    g = _graph(code)
    assert (g.n, g.m, g.nnz) == (code.n, code.m, code.nnz)
    lab = code.labels()
    assert g.max_cdeg == (lab > 0).sum(1).max() and g.max_vdeg == (lab > 0).sum(0).max()
    c, q = g.edges()
    rows, cols = np.nonzero(lab)
    assert np.array_equal(c, rows) and np.array_equal(q, cols)
    assert g.device_bytes() > 0 and g.device_bytes() % 256 == 0


def _err(fn):
    from paper_2407_11523_amd import BP4Error
    with pytest.raises(BP4Error) as ei:
        fn()
    return ei.value.name


def test_graph_create_errors(lib):
    from paper_2407_11523_amd import Graph
    code = qecgen.planar(3)
    assert _err(lambda: Graph(code.hx * 2, code.hz, upload=False)) == "EINVAL"
    z = np.zeros((0, 4), np.uint8)
    assert _err(lambda: Graph(z, z, upload=False)) == "EINVAL"
    hx = code.hx.copy()
    hz = code.hz.copy()
    hx[0] = 0
    hz[0] = 0
    assert _err(lambda: Graph(hx, hz, upload=False)) == "EINVAL"          # empty check
    hx = np.hstack([code.hx, np.zeros((code.m, 1), np.uint8)])
    hz = np.hstack([code.hz, np.zeros((code.m, 1), np.uint8)])
    assert _err(lambda: Graph(hx, hz, upload=False)) == "EINVAL"          # qubit in no check
    a = np.array([[1, 0], [0, 1]], np.uint8)
    b = np.array([[0, 0], [1, 0]], np.uint8)
    assert _err(lambda: Graph(a, b, upload=False)) == "ENONCOMM"
    Graph(a, b, upload=False, allow_anticommuting=True)                    # allowed with the flag
    wide = np.ones((1, 9), np.uint8)                                      # a check of degree 9
    assert _err(lambda: Graph(wide, np.zeros_like(wide), upload=False)) == "EDEGREE"
    deep = np.ones((8, 1), np.uint8)                                      # a qubit of degree 8
    assert _err(lambda: Graph(deep, np.zeros_like(deep), upload=False)) == "EDEGREE"
    big = np.ones((1, 16384), np.uint8)
    assert _err(lambda: Graph(big, np.zeros_like(big), upload=False)) == "EUNSUPPORTED"


def test_param_validation_before_launch(lib):
    from paper_2407_11523_amd import Params
    g = _graph(qecgen.toric(4))
    ok = Params(variant="ewainit", alpha=0.5)
    assert g.workspace_bytes(ok, 100) >= 4
    for bad in (Params(variant="ewainit", alpha=1.5), Params(variant="momentum", alpha=-0.1),
                Params(variant="momentum", gamma=1.0), Params(variant="adagrad", alpha=0.0),
                Params(variant="adagrad", alpha=5.0, eps=0.0), Params(max_iter=0),
                Params(llr_clamp=0.0), Params(llr_clamp=float("inf"))):
        assert _err(lambda: g.workspace_bytes(bad, 10)) == "EINVAL"


def test_decode_rejects_bad_pointers_without_gpu(lib):
    from paper_2407_11523_amd import Params, _lib
    g = _graph(qecgen.toric(4))
    cp = Params().c()
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: validation fails first
    rc = lib.bp4_decode(g.handle, null, ctypes.byref(cp), 10, fake, fake, fake, fake, fake, fake, 256, null)
    assert rc == -1
    rc = lib.bp4_decode(g.handle, fake, ctypes.byref(cp), 10, null, fake, fake, fake, fake, fake, 256, null)
    assert rc == -1
    rc = lib.bp4_decode(g.handle, fake, ctypes.byref(cp), 10, fake, fake, fake, fake, fake, fake, 8, null)
    assert rc == -4
    rc = lib.bp4_decode(g.handle, fake, ctypes.byref(cp), -1, fake, fake, fake, fake, fake, fake, 256, null)
    assert rc == -1
    tune = _lib.Tuning(48)
    rc = lib.bp4_decode_ex(g.handle, fake, ctypes.byref(cp), ctypes.byref(tune), 10, fake, fake, fake, fake,
                           fake, null, null, null, fake, 256, null)
    assert rc == -1
    tune = _lib.Tuning(0, 0, 7)                       # unknown kernel
    rc = lib.bp4_decode_ex(g.handle, fake, ctypes.byref(cp), ctypes.byref(tune), 10, fake, fake, fake, fake,
                           fake, null, null, null, fake, 1 << 30, null)
    assert rc == -1
    tune = _lib.Tuning(64, 0, 2)                      # group size with the SOA kernel
    rc = lib.bp4_decode_ex(g.handle, fake, ctypes.byref(cp), ctypes.byref(tune), 10, fake, fake, fake, fake,
                           fake, null, null, null, fake, 1 << 30, null)
    assert rc == -1
    tune = _lib.Tuning(0, 0, 1, 4096)                 # SOA lanes with the LDS kernel
    rc = lib.bp4_decode_ex(g.handle, fake, ctypes.byref(cp), ctypes.byref(tune), 10, fake, fake, fake, fake,
                           fake, null, null, null, fake, 1 << 30, null)
    assert rc == -1
    tune = _lib.Tuning(0, 0, 2)                       # SOA workspace too small
    rc = lib.bp4_decode_ex(g.handle, fake, ctypes.byref(cp), ctypes.byref(tune), 10, fake, fake, fake, fake,
                           fake, null, null, null, fake, 4096, null)
    assert rc == -4
    assert b"SOA" in lib.bp4_last_error()
    t = (ctypes.c_uint32 * 3)(2 ** 31, 2 ** 31, 1)
    rc = lib.bp4_sample(g.handle, fake, 10, 0, t, 1, 0, fake, fake, null)
    assert rc == -1
    g2 = _graph(qecgen.toric(4))
    from paper_2407_11523_amd import Graph
    g3 = Graph(qecgen.toric(4).hx, qecgen.toric(4).hz, upload=False)   # no logicals
    rc = lib.bp4_bookkeep(g3.handle, fake, 10, fake, fake, fake, fake, null)
    assert rc == -1
    assert b"logical" in lib.bp4_last_error()
    del g2


def test_mixed_and_plain_validation_without_gpu(lib):
    from paper_2407_11523_amd import Params, _lib
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(1 << 20)
    b = ctypes.c_size_t()
    assert lib.bp4_mixed_workspace_bytes(0, ctypes.byref(b)) == -1
    assert lib.bp4_mixed_workspace_bytes(17, ctypes.byref(b)) == -1
    assert lib.bp4_mixed_workspace_bytes(11, ctypes.byref(b)) == 0 and b.value >= 4 * 11
    arr = (_lib.CodeBatch * 2)()
    assert lib.bp4_decode_mixed(2, arr, fake, 256, null) == -1          # NULL graphs
    assert lib.bp4_decode_mixed(0, arr, fake, 256, null) == -1
    assert lib.bp4_decode_mixed(2, arr, fake, 16, null) == -4           # workspace too small
    g = _graph(qecgen.toric(4))
    cp = Params(variant="momentum", alpha=0.5).c()
    arr[0] = _lib.CodeBatch(g.handle.value, fake.value, cp, 10, fake.value, fake.value, fake.value, fake.value,
                            fake.value, 0, 600)
    arr[1] = arr[0]
    assert lib.bp4_decode_mixed(2, arr, fake, 256, null) == -1          # block_shots above 512
    assert b"block_shots" in lib.bp4_last_error()
    arr[0].group_lanes, arr[0].block_shots = 64, 2
    arr[1] = arr[0]
    assert lib.bp4_decode_mixed(2, arr, fake, 256, null) == -1          # block_shots with a wave group
    assert lib.bp4_plain_workspace_bytes(g.handle, ctypes.byref(cp), 1000, ctypes.byref(b)) == 0
    assert b.value >= 1000 * (g.nnz * 4 + 2 * 3 * g.n * 4 + g.n)
    it = ctypes.c_int32()
    assert lib.bp4_decode_plain(g.handle, fake, ctypes.byref(cp), 1000, fake, fake, fake, fake, fake, fake, 64,
                                null, ctypes.byref(it)) == -4


def test_large_codes_take_the_hbm_kernels(lib):
    """Codes whose LDS image exceeds the automatic limit run from HBM.  The two-phase SOA
    kernel's workspace holds every message and qubit state per resident lane and grows
    with the variant; the automatic choice for every flooding variant is the single-pass
    kernel, whose workspace is two 64-column records per workgroup in
    flight (32 wavefronts per CU; 4 message words per check, 3 posterior words per
    qubit, 3 more for the Momentum and AdaGrad accumulators)."""
    from paper_2407_11523_amd import Graph, Params
    c = qecgen.planar(31)
    g = Graph(c.hx, c.hz, upload=False)
    m, n = c.hx.shape
    shots = 1 << 18
    sizes = {}
    for v in ("bp", "ewainit", "momentum", "adagrad"):
        prm = Params(variant=v, alpha=0.5 if v != "adagrad" else 5.0)
        b = ctypes.c_size_t()
        assert lib.bp4_soa_workspace_bytes(g.handle, ctypes.byref(prm.c()), shots, 0, ctypes.byref(b)) == 0
        sizes[v] = b.value
        items = 4 * m + 3 * n + (3 * n if v in ("momentum", "adagrad") else 0)
        head = 256 + (4 * m * 4 + 255) // 256 * 256
        # 32 wavefronts per CU: 512 workgroups of 16 in flight, 1024 of 8, or one per 64 shots
        want = head + 512 * 2 * items * 256
        assert g.gather_workspace_bytes(prm, shots) == want
        assert g.workspace_bytes(prm, shots) == want
        assert g.gather_workspace_bytes(prm, 100) == head + 2 * 2 * items * 256
        assert g.gather_workspace_bytes(prm, shots, 8) == head + 1024 * 2 * items * 256
    # the serial schedule and AEWA (EWAInit's records) take the single-pass kernel too
    ser = Params(variant="ewainit", alpha=0.5, serial=True)
    b = ctypes.c_size_t()
    assert g.workspace_bytes(ser, shots) == g.gather_workspace_bytes(ser, shots) == head + 512 * 2 * (4 * m + 3 * n) * 256
    ae = Params(variant="aewa", alpha=0.5, alpha_last=0.9, alpha_steps=3)
    assert g.workspace_bytes(ae, shots) == g.gather_workspace_bytes(ae, shots) == head + 512 * 2 * (4 * m + 3 * n) * 256
    prm = Params(variant="bp")
    for bad in (-1, 2, 32):
        assert lib.bp4_gather_workspace_bytes(g.handle, ctypes.byref(prm.c()), shots, bad, ctypes.byref(b)) == -1
    assert b"gather_waves" in lib.bp4_last_error() or b"negative" in lib.bp4_last_error()
    assert lib.bp4_gather_workspace_bytes(g.handle, ctypes.byref(prm.c()), -1, 0, ctypes.byref(b)) == -1
    # BP: messages (nnz + 1 slots) + decisions + syndrome bits; EWAInit adds Q; the others add a second state
    lanes = shots
    # two records per lane (running and packed), plus decisions
    assert sizes["bp"] >= 2 * (7320 + 59) * lanes * 4 + 1861 * lanes
    assert sizes["ewainit"] - sizes["bp"] >= 2 * 3 * 1861 * lanes * 4
    assert sizes["momentum"] - sizes["ewainit"] >= 2 * 3 * 1861 * lanes * 4
    assert sizes["adagrad"] == sizes["momentum"]
    # fewer lanes in flight: proportionally smaller
    b = ctypes.c_size_t()
    assert lib.bp4_soa_workspace_bytes(g.handle, ctypes.byref(prm.c()), shots, 1 << 14, ctypes.byref(b)) == 0
    assert b.value * 15 < sizes["bp"] < b.value * 17
    assert lib.bp4_soa_workspace_bytes(g.handle, ctypes.byref(prm.c()), shots, -1, ctypes.byref(b)) == -1
    # the small codes keep the LDS kernel's 256-byte workspace
    s = qecgen.planar(13)
    gs = Graph(s.hx, s.hz, upload=False)
    assert gs.workspace_bytes(Params(variant="ewainit", alpha=0.5), shots) == 256


def test_gather_kernel_validation_without_gpu(lib):
    """The single-pass HBM kernel's argument checks run before any launch: no verification
    outputs, gather_waves in {0, 4, 8, 16}, its own workspace
    size, and its tuning field excludes the LDS and SOA ones."""
    from paper_2407_11523_amd import Graph, Params, _lib
    c = qecgen.toric(32)
    g = Graph(c.hx, c.hz, upload=False)
    fake = ctypes.c_void_p(1 << 20)
    null = ctypes.c_void_p(0)
    cp = Params(variant="ewainit", alpha=0.6).c()
    need = g.gather_workspace_bytes(Params(variant="ewainit", alpha=0.6), 1000)

    def dec(tune, q=null, ws_bytes=need, params=cp):
        return lib.bp4_decode_ex(g.handle, fake, ctypes.byref(params), ctypes.byref(tune), 1000, fake, fake, fake,
                                 fake, fake, q, q, q, fake, ws_bytes, null)

    assert dec(_lib.Tuning(0, 0, 3), q=fake) == -6                      # verification outputs
    assert b"q_out" in lib.bp4_last_error()
    assert dec(_lib.Tuning(0, 0, 3), ws_bytes=need - 1) == -4           # workspace too small
    assert dec(_lib.Tuning(0, 0, 3, 0, 0, 0, 5)) == -1                  # gather_waves 5
    assert dec(_lib.Tuning(0, 0, 2, 0, 0, 0, 8)) == -1                  # gather_waves with SOA
    assert dec(_lib.Tuning(0, 0, 1, 0, 0, 0, 8)) == -1                  # gather_waves with LDS
    assert dec(_lib.Tuning(0, 0, 0, 1024, 0, 0, 8)) == -1               # SOA and gather fields together
    assert dec(_lib.Tuning(64, 0, 3)) == -1                             # LDS field with the gather kernel
    assert dec(_lib.Tuning(0, 0, 3, 0, 0, 0, 0, 1)) == -1               # reserved
    ser = Params(variant="ewainit", alpha=0.6, serial=True)
    need_ser = g.gather_workspace_bytes(ser, 1000)
    assert dec(_lib.Tuning(0, 0, 3), params=ser.c(), ws_bytes=need_ser - 1) == -4   # serial runs: its workspace
    ae = Params(variant="aewa", alpha=0.5, alpha_last=0.9, alpha_steps=3)
    need_ae = g.gather_workspace_bytes(ae, 1000)
    assert dec(_lib.Tuning(0, 0, 3), params=ae.c(), ws_bytes=need_ae - 1) == -4   # AEWA runs: its workspace
    # wide graphs: LDS kernel only
    bb = qecgen.bb(72)
    gw = Graph(bb.hx, bb.hz, upload=False)
    assert lib.bp4_decode_ex(gw.handle, fake, ctypes.byref(cp), ctypes.byref(_lib.Tuning(0, 0, 3)), 1000, fake,
                             fake, fake, fake, fake, null, null, null, fake, 1 << 30, null) == -6


def test_mixed_rejects_soa_only_codes(lib):
    from paper_2407_11523_amd import Graph, Params, _lib
    c = qecgen.toric(32)
    g = Graph(c.hx, c.hz, upload=False)
    fake = ctypes.c_void_p(1 << 20)
    arr = (_lib.CodeBatch * 1)()
    arr[0] = _lib.CodeBatch(g.handle.value, fake.value, Params(variant="ewainit", alpha=0.5).c(), 10, fake.value,
                            fake.value, fake.value, fake.value, fake.value, 0, 0)
    assert lib.bp4_decode_mixed(1, arr, fake, 4096, None) == -6
    assert b"SOA" in lib.bp4_last_error()


EW = 3   # BP4_EWAINIT


def test_unrolled_sizes_and_validation(lib):
    from paper_2407_11523_amd import Graph
    c = qecgen.planar(9)
    g = Graph(c.hx, c.hz, upload=False)
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.bp4_unrolled_sizes(g.handle, EW, 32, 8, 1 << 16, ctypes.byref(a), ctypes.byref(b)) == 0
    state = (544 + 3 * 145) * 4 * (1 << 16)          # messages + posteriors per shot, 65,536 shots
    assert a.value == 4 * state                       # checkpoints at t = 0, 8, 16, 24
    assert b.value >= 9 * state                       # one segment: its first state and 8 more
    a2, b2 = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.bp4_unrolled_sizes(g.handle, EW, 32, 32, 1 << 16, ctypes.byref(a2), ctypes.byref(b2)) == 0
    assert a2.value == state and b2.value > b.value   # fewer checkpoints, longer segment
    for T, K, shots in ((0, 8, 10), (8, 0, 10), (8, 4, 0)):
        assert lib.bp4_unrolled_sizes(g.handle, EW, T, K, shots, ctypes.byref(a), ctypes.byref(b)) == -1
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(1 << 20)
    # undersized buffers and bad arguments fail before any launch
    rc = lib.bp4_unrolled_forward(g.handle, fake, EW, 32, 8, 30.0, 1 << 16, fake, fake, fake, fake, fake, null,
                                  fake, 1024, fake, 1 << 40, null)
    assert rc == -4
    rc = lib.bp4_unrolled_forward(g.handle, fake, EW, 32, 8, 0.0, 1 << 16, fake, fake, fake, fake, fake, null,
                                  fake, 1 << 40, fake, 1 << 40, null)
    assert rc == -1
    rc = lib.bp4_unrolled_backward(g.handle, fake, EW, 32, 8, 30.0, 1 << 16, fake, fake, fake, null, null, fake,
                                   1 << 40, fake, fake, fake, 1 << 40, null)
    assert rc == -1
    rc = lib.bp4_unrolled_backward(g.handle, fake, EW, 32, 8, 30.0, 1 << 16, fake, fake, fake, fake, null, fake,
                                   1 << 40, fake, fake, fake, 64, null)
    assert rc == -4
    # Momentum: a state holds Q, g and M (9 words per qubit after the messages); undersized
    # buffers fail before any launch
    assert lib.bp4_unrolled_sizes(g.handle, 1, 32, 8, 1 << 16, ctypes.byref(a), ctypes.byref(b)) == 0
    assert a.value == 4 * (544 + 9 * 145) * 4 * (1 << 16)
    rc = lib.bp4_unrolled_forward(g.handle, fake, 1, 32, 8, 30.0, 1 << 16, fake, fake, fake, fake, fake, null,
                                  fake, 1024, fake, 1 << 40, null)
    assert rc == -4
    rc = lib.bp4_unrolled_backward(g.handle, fake, 1, 32, 8, 30.0, 1 << 16, fake, fake, fake, fake, null, fake,
                                   1 << 40, fake, fake, fake, 64, null)
    assert rc == -4
    # the unrolled path is built for EWAInit and Momentum: the others are refused before any launch
    for variant in (0, 2, 4):
        assert lib.bp4_unrolled_sizes(g.handle, variant, 32, 8, 1 << 16, ctypes.byref(a), ctypes.byref(b)) == -6
        rc = lib.bp4_unrolled_forward(g.handle, fake, variant, 32, 8, 30.0, 1 << 16, fake, fake, fake, fake, fake,
                                      null, fake, 1 << 40, fake, 1 << 40, null)
        assert rc == -6
        rc = lib.bp4_unrolled_backward(g.handle, fake, variant, 32, 8, 30.0, 1 << 16, fake, fake, fake, fake, null,
                                       fake, 1 << 40, fake, fake, fake, 1 << 40, null)
        assert rc == -6
    assert lib.bp4_unrolled_sizes(g.handle, 7, 32, 8, 1 << 16, ctypes.byref(a), ctypes.byref(b)) == -1


def test_unrolled_binding_validates_inputs(lib):
    # wrong shapes, dtypes or devices are refused by the binding before the library is called
    import torch
    from paper_2407_11523_amd import BP4Error, Graph, unrolled_forward
    c = qecgen.planar(3)
    g = Graph(c.hx, c.hz, upload=False)
    g.dev = torch.zeros(g.device_bytes(), dtype=torch.uint8)      # a host stand-in: never launched
    T = 4
    ok = dict(alpha=torch.zeros(T), prior=torch.zeros(c.n, 3), synd=torch.zeros(8, c.m, dtype=torch.uint8),
              err=torch.zeros(8, c.n, dtype=torch.uint8))
    bad = [dict(alpha=torch.zeros(T + 1)), dict(prior=torch.zeros(c.n, 2)),
           dict(synd=torch.zeros(8, c.m, dtype=torch.int32)), dict(synd=torch.zeros(8, c.m + 1, dtype=torch.uint8)),
           dict(err=torch.zeros(7, c.n, dtype=torch.uint8)), dict(err=torch.zeros(8, c.n)),
           dict(synd=torch.zeros(0, c.m, dtype=torch.uint8), err=torch.zeros(0, c.n, dtype=torch.uint8)),
           dict(alpha=torch.zeros(T, dtype=torch.int64))]
    for b in bad:
        kw = dict(ok, **b)
        with pytest.raises(BP4Error):
            unrolled_forward(g, kw["alpha"], kw["prior"], kw["synd"], kw["err"], T)
    # Momentum takes (alpha_t, gamma_t) per iteration, [T, 2]; variants without an unrolled
    # build are refused
    for params, variant in ((torch.zeros(T), "momentum"), (torch.zeros(T, 3), "momentum"),
                            (torch.zeros(T, 2), "ewainit"), (torch.zeros(T), "adagrad"), (torch.zeros(T), "bp")):
        with pytest.raises(BP4Error):
            unrolled_forward(g, params, ok["prior"], ok["synd"], ok["err"], T, variant=variant)


def test_prior_llr_validation_without_gpu(lib):
    from paper_2407_11523_amd import BP4Error, prior_llr
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(1 << 20)
    assert lib.bp4_prior_llr(0, fake, fake, null) == -1
    assert lib.bp4_prior_llr(16384, fake, fake, null) == -1
    assert lib.bp4_prior_llr(4, null, fake, null) == -1
    assert lib.bp4_prior_llr(4, fake, null, null) == -1
    for probs in (np.zeros((3, 3)), np.full((2, 3), 0.4), np.array([[0.1, np.nan, 0.1]]), np.full((2, 2), 0.1),
                  np.array([[0.1, -0.01, 0.1]])):
        with pytest.raises(BP4Error):
            prior_llr(probs, device="cpu")


def test_aewa_parameter_validation(lib):
    from paper_2407_11523_amd import Graph, Params
    g = Graph(qecgen.planar(5).hx, qecgen.planar(5).hz, upload=False)
    ok = Params(variant="aewa", alpha=1.0, alpha_last=0.0, alpha_steps=11)
    assert g.workspace_bytes(ok, 10) == 256
    for bad in (Params(variant="aewa", alpha_steps=0), Params(variant="aewa", alpha_steps=65),
                Params(variant="aewa", alpha_last=1.5), Params(variant="aewa", alpha=-0.1),
                Params(variant="aewa", stop_on_syndrome=False)):
        assert _err(lambda: g.workspace_bytes(bad, 10)) == "EINVAL"
    # the other variants ignore the AEWA fields
    assert g.workspace_bytes(Params(variant="ewainit", alpha=0.5, alpha_steps=0, alpha_last=7.0), 10) == 256


def test_lane_mapping_validation_and_layout(lib):
    """Block slots: the layout holds S regions (each with syndrome bytes and a header),
    group_lanes 128 / 256 / 512 alone are 4 / 2 / 1 slots of a 512-lane workgroup, and
    invalid mappings are rejected before anything is enqueued."""
    from paper_2407_11523_amd import Params, _lib
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(1 << 20)
    g = _graph(qecgen.planar(9))
    cp = Params(variant="ewainit", alpha=0.5).c()

    def layout(G, S):
        b = ctypes.c_size_t()
        rc = lib.bp4_lds_layout_bytes(g.handle, ctypes.byref(cp), G, S, ctypes.byref(b))
        return rc, b.value

    rc1, b1 = layout(512, 0)
    rc2, b2 = layout(0, 1)
    assert rc1 == 0 and rc2 == 0 and b1 == b2
    assert layout(256, 0) == layout(512, 2) == layout(0, 2)
    assert layout(128, 0) == layout(0, 4)
    region = layout(0, 2)[1] - b2
    assert layout(0, 3)[1] == b2 + 2 * region and layout(0, 4)[1] == b2 + 3 * region
    # a region holds the messages (four slot-major slots per qubit and the padding
    # slot), posteriors, decisions, syndrome bytes and a header
    assert region >= 4 * (4 * g.n + 1 + 3 * g.n) + g.n + g.m
    assert layout(0, 0)[0] == -1           # no mapping
    assert layout(64, 2)[0] == -1          # block_shots with a wave group
    assert layout(0, 513)[0] == -1
    assert layout(1024, 0)[0] == -1
    assert layout(48, 0)[0] == -1
    # more than 64 check items per lane (392 checks: 83 shots fit 64 x 512 items)
    big = _graph(qecgen.toric(14))
    b = ctypes.c_size_t()
    assert lib.bp4_lds_layout_bytes(big.handle, ctypes.byref(cp), 0, 83, ctypes.byref(b)) == 0
    assert lib.bp4_lds_layout_bytes(big.handle, ctypes.byref(cp), 0, 84, ctypes.byref(b)) == -1
    for G, S in ((64, 1), (0, 600), (32, 4)):
        tune = _lib.Tuning(G, 0, 0, 0, 0, S)
        rc = lib.bp4_decode_ex(g.handle, fake, ctypes.byref(cp), ctypes.byref(tune), 10, fake, fake, fake, fake,
                               fake, null, null, null, fake, 256, null)
        assert rc == -1, (G, S)
    tune = _lib.Tuning(0, 0, 2, 0, 0, 2)   # block_shots with the SOA kernel
    rc = lib.bp4_decode_ex(g.handle, fake, ctypes.byref(cp), ctypes.byref(tune), 10, fake, fake, fake, fake,
                           fake, null, null, null, fake, 1 << 30, null)
    assert rc == -1


def test_wide_graphs_route_to_the_flooding_lds_kernel(lib):
    """Degree-6 codes build as wide graphs; the paths that need narrow graphs refuse them
    before anything is enqueued."""
    from paper_2407_11523_amd import Graph, Params, _lib
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(1 << 20)
    for c in (qecgen.bb(72), qecgen.chamon(2)):
        g = Graph(c.hx, c.hz, c.lx, c.lz, upload=False)
        n, m, nnz, dc, dv = (ctypes.c_int32() for _ in range(5))
        assert lib.bp4_graph_info(g.handle, *(ctypes.byref(x) for x in (n, m, nnz, dc, dv))) == 0
        assert (n.value, m.value, dc.value, dv.value) == (c.n, c.m, 6, 6)
        cp = Params(variant="ewainit", alpha=0.5).c()
        b = ctypes.c_size_t()
        assert lib.bp4_workspace_bytes(g.handle, ctypes.byref(cp), 1000, ctypes.byref(b)) == 0 and b.value == 256
        # the wide layout holds 8 edge words per check and a label word per qubit
        assert lib.bp4_lds_layout_bytes(g.handle, ctypes.byref(cp), 64, 0, ctypes.byref(b)) == 0
        assert b.value >= 4 * (8 * c.m + 5 * c.n)
        tune = _lib.Tuning(0, 0, 2)                                       # the SOA kernel
        rc = lib.bp4_decode_ex(g.handle, fake, ctypes.byref(cp), ctypes.byref(tune), 10, fake, fake, fake, fake,
                               fake, null, null, null, fake, 1 << 30, null)
        assert rc == -6, rc                                                # EUNSUPPORTED
        sp = Params(variant="ewainit", alpha=0.5, serial=True).c()
        # the serial schedule runs on the LDS kernel's wide build: its workspace is checked
        # before anything runs; on the SOA kernel it is refused
        rc = lib.bp4_decode(g.handle, fake, ctypes.byref(sp), 10, fake, fake, fake, fake, fake, fake, 0, null)
        assert rc == -4, rc                                                # EWORKSPACE
        rc = lib.bp4_decode_ex(g.handle, fake, ctypes.byref(sp), ctypes.byref(tune), 10, fake, fake, fake, fake,
                               fake, null, null, null, fake, 1 << 30, null)
        assert rc == -6, rc                                                # EUNSUPPORTED
        it = ctypes.c_int32()
        # the plain decoder takes wide graphs: its workspace is checked before anything runs
        assert lib.bp4_decode_plain(g.handle, fake, ctypes.byref(cp), 10, fake, fake, fake, fake, fake, fake,
                                    0, null, ctypes.byref(it)) == -4
        s1, s2 = ctypes.c_size_t(), ctypes.c_size_t()
        assert lib.bp4_unrolled_sizes(g.handle, EW, 4, 2, 64, ctypes.byref(s1), ctypes.byref(s2)) == 0
    # a mixed launch may combine wide and narrow codes; its buffers are still checked first
    gw = Graph(qecgen.bb(72).hx, qecgen.bb(72).hz, upload=False)
    gn = Graph(qecgen.toric(4).hx, qecgen.toric(4).hz, upload=False)
    cp = Params(variant="ewainit", alpha=0.5).c()
    arr = (_lib.CodeBatch * 2)()
    arr[0] = _lib.CodeBatch(gw.handle.value, fake.value, cp, 10, fake.value, fake.value, fake.value, fake.value,
                            fake.value, 0, 0)
    arr[1] = _lib.CodeBatch(gn.handle.value, fake.value, cp, 10, fake.value, fake.value, None, fake.value,
                            fake.value, 0, 0)
    assert lib.bp4_decode_mixed(2, arr, fake, 256, null) == -1                         # EINVAL: NULL est


def test_graph_set_coords(lib):
    """Qubit coordinates re-order the single-pass kernel's walk only: any integer layout
    is accepted for a narrow graph, the image size does not change, wide graphs (no
    single-pass kernel) and NULL arguments are refused."""
    from paper_2407_11523_amd import BP4Error, Graph
    i32p = ctypes.POINTER(ctypes.c_int32)
    code = qecgen.planar(7)
    g = Graph(code.hx, code.hz, code.lx, code.lz, upload=False)
    before = g.device_bytes()
    xy = np.ascontiguousarray(code.coords, dtype=np.int32)
    assert lib.bp4_graph_set_coords(None, xy.ctypes.data_as(i32p)) == -1
    assert lib.bp4_graph_set_coords(g.handle, None) == -1
    assert lib.bp4_graph_set_coords(g.handle, xy.ctypes.data_as(i32p)) == 0
    assert g.device_bytes() == before
    # every qubit at one point, or a random layout: still a valid walk
    same = np.zeros((code.n, 2), np.int32)
    assert lib.bp4_graph_set_coords(g.handle, same.ctypes.data_as(i32p)) == 0
    g.set_coords(np.random.default_rng(1).integers(-50, 50, (code.n, 2)))
    with pytest.raises(BP4Error):
        g.set_coords(xy[:-1])
    wide = Graph(qecgen.bb(72).hx, qecgen.bb(72).hz, upload=False)
    xyw = np.zeros((wide.n, 2), np.int32)
    assert lib.bp4_graph_set_coords(wide.handle, xyw.ctypes.data_as(i32p)) == -6
    # the lattice families carry their layouts; each check's qubits sit within two units
    for fam, size, per in (("planar", 5, None), ("toric", 6, 12), ("xzzx", 5, 5)):
        c = qecgen.make(fam, size)
        assert c.coords.shape == (c.n, 2) and len({tuple(p) for p in c.coords}) == c.n
        H = (c.hx | c.hz).astype(bool)
        for r in range(c.m):
            pts = c.coords[np.nonzero(H[r])[0]]
            d = np.abs(pts[:, None, :] - pts[None, :, :])
            if per:
                d = np.minimum(d, per - d)
            assert int(d.max()) <= 2, (fam, r)
