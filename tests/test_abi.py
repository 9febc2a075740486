"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/mpid.h declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpid.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(id_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2012_00706_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2012_00706_amd.build import build_library
        build_library()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert {"id_factor", "id_solve_T", "id_reconstruct", "id_backward",
            "id_workspace_size", "id_status_string"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_header(lib):
    from paper_2012_00706_amd import _lib
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_status_strings(lib):
    from paper_2012_00706_amd import C
    for key in ("ID_OK", "ID_ERR_ARG", "ID_ERR_WORKSPACE", "ID_INFO_SINGULAR"):
        s = lib.id_status_string(C[key]).decode()
        assert s and s != "unknown code"
    assert lib.id_status_string(12345).decode() == "unknown code"


def test_workspace_size_host_logic(lib):
    from paper_2012_00706_amd import C, make_opts
    o = make_opts(tol=1e-3, prec="mixed_bf16")
    s1 = lib.id_workspace_size(20000, 2000, C["ID_F32"], ctypes.byref(o))
    # two fp32 working copies dominate
    assert s1 >= 2 * 20000 * 2048 * 4
    o64 = make_opts(tol=1e-3, prec="f64")
    s2 = lib.id_workspace_size(20000, 2000, C["ID_F32"], ctypes.byref(o64))
    assert s2 > s1
    bad = make_opts(k=3)
    bad.nb = 99
    assert lib.id_workspace_size(10, 10, C["ID_F32"], ctypes.byref(bad)) == 0
    assert lib.id_workspace_size(-1, 10, C["ID_F32"], ctypes.byref(o)) == 0
    assert lib.id_workspace_size(10, 10, 7, ctypes.byref(o)) == 0


def test_argument_errors_return_before_any_device_call(lib):
    from paper_2012_00706_amd import C, make_opts
    o = make_opts(k=2)
    k = ctypes.c_int64(0)
    info = ctypes.c_int32(0)
    # null A
    rc = lib.id_factor(None, C["ID_F64"], 10, 5, 10, ctypes.byref(o), None, 0, None, None, 2,
                       ctypes.byref(k), ctypes.byref(info), None)
    assert rc == C["ID_ERR_ARG"]
    # bad dtype
    rc = lib.id_factor(None, 9, 10, 5, 10, ctypes.byref(o), None, 0, None, None, 2,
                       ctypes.byref(k), ctypes.byref(info), None)
    assert rc == C["ID_ERR_DTYPE"]
    # lda < m
    fake = ctypes.c_void_p(0x1000)
    rc = lib.id_factor(fake, C["ID_F64"], 10, 5, 3, ctypes.byref(o), fake, 1 << 30, fake, fake, 2,
                       ctypes.byref(k), ctypes.byref(info), None)
    assert rc == C["ID_ERR_ARG"]
    # workspace too small
    rc = lib.id_factor(fake, C["ID_F64"], 10, 5, 10, ctypes.byref(o), fake, 16, fake, fake, 2,
                       ctypes.byref(k), ctypes.byref(info), None)
    assert rc == C["ID_ERR_WORKSPACE"]
    # solve_T: n < k
    rc = lib.id_solve_T(fake, 5, 6, 5, fake, 6, fake, None)
    assert rc == C["ID_ERR_ARG"]
    # reconstruct: k > n
    rc = lib.id_reconstruct(fake, C["ID_F32"], 4, 3, 4, fake, 5, fake, 5, fake, 4, 0, None)
    assert rc == C["ID_ERR_ARG"]
    rc = lib.id_backward(fake, C["ID_F32"], 4, 3, 4, fake, 5, fake, 5, None, 1, None, 1, None, 4,
                         fake, 4, fake, 1 << 20, ctypes.byref(info), None)
    assert rc == C["ID_ERR_ARG"]
    # backward: a supplied R11 with ldrb < k
    rc = lib.id_backward(fake, C["ID_F32"], 8, 6, 8, fake, 3, fake, 3, fake, 2, None, 1, None, 8,
                         fake, 8, fake, 1 << 20, ctypes.byref(info), None)
    assert rc == C["ID_ERR_ARG"]
    assert lib.id_backward_workspace_size(4, 3, 5) == 0
    # sketch: ldo < m, ldy < l, small workspace, bad dtype
    ws = lib.id_sketch_workspace_size(8, 100, 10)
    assert ws > 0 and lib.id_sketch_workspace_size(-1, 100, 10) == 0
    rc = lib.id_sketch(fake, C["ID_F32"], 100, 10, 100, fake, 8, 99, fake, 8, fake, ws, None)
    assert rc == C["ID_ERR_ARG"]
    rc = lib.id_sketch(fake, C["ID_F32"], 100, 10, 100, fake, 8, 100, fake, 7, fake, ws, None)
    assert rc == C["ID_ERR_ARG"]
    rc = lib.id_sketch(fake, C["ID_F32"], 100, 10, 100, fake, 8, 100, fake, 8, fake, ws - 8, None)
    assert rc == C["ID_ERR_WORKSPACE"]
    rc = lib.id_sketch(fake, 7, 100, 10, 100, fake, 8, 100, fake, 8, fake, ws, None)
    assert rc == C["ID_ERR_DTYPE"]


def test_options_validation():
    from paper_2012_00706_amd import make_opts
    with pytest.raises(ValueError):
        make_opts()
    with pytest.raises(ValueError):
        make_opts(k=3, prec="fp8")
    with pytest.raises(ValueError):
        make_opts(k=3, rule="nope")


def test_noalloc_host_checks(lib):
    """id_factor_noalloc refuses, before any device call, what does not fit
    its static scratch and the flags it does not take."""
    from paper_2012_00706_amd import C, make_opts
    assert lib.id_noalloc_scratch_bytes() == C["ID_NOALLOC_SCRATCH_MB"] << 20
    k = ctypes.c_int64(0)
    info = ctypes.c_int32(0)
    fake = ctypes.c_void_p(0x1000)
    o = make_opts(tol=1e-3, prec="mixed_bf16x3")
    # 20000 x 2000 fp32 needs about 362 MiB of workspace
    assert lib.id_workspace_size(20000, 2000, C["ID_F32"], ctypes.byref(o)) > \
        lib.id_noalloc_scratch_bytes()
    rc = lib.id_factor_noalloc(fake, C["ID_F32"], 20000, 2000, 20000, ctypes.byref(o), fake, fake,
                               2000, ctypes.byref(k), ctypes.byref(info), None)
    assert rc == C["ID_ERR_SCRATCH"]
    assert lib.id_status_string(rc).decode() != "unknown code"
    g = make_opts(tol=1e-3, gram=True)
    rc = lib.id_factor_noalloc(fake, C["ID_F64"], 100, 10, 100, ctypes.byref(g), fake, fake, 10,
                               ctypes.byref(k), ctypes.byref(info), None)
    assert rc == C["ID_ERR_UNSUPPORTED"]
    rc = lib.id_factor_noalloc(fake, 9, 100, 10, 100, ctypes.byref(o), fake, fake, 10,
                               ctypes.byref(k), ctypes.byref(info), None)
    assert rc == C["ID_ERR_DTYPE"]


def test_round_and_flag_host_checks(lib):
    """id_round and the simulated-precision flags: argument errors before any
    device call."""
    from paper_2012_00706_amd import C, make_opts
    fake = ctypes.c_void_p(0x1000)
    assert lib.id_round(fake, 4, 4, 4, 3, None) == C["ID_ERR_ARG"]      # unknown mode
    assert lib.id_round(fake, 4, 4, 3, 1, None) == C["ID_ERR_ARG"]      # ld < rows
    assert lib.id_round(None, 0, 5, 1, 2, None) == C["ID_OK"]           # empty
    both = make_opts(k=3)
    both.flags = C["ID_FLAG_ROUND_F32"] | C["ID_FLAG_ROUND_F16"]
    assert lib.id_workspace_size(10, 10, C["ID_F32"], ctypes.byref(both)) == 0
    g = make_opts(tol=1e-3, prec="mixed_f32", gram=True, round_to="f32")
    k = ctypes.c_int64(0)
    info = ctypes.c_int32(0)
    ws = lib.id_workspace_size(100, 10, C["ID_F64"], ctypes.byref(g))
    rc = lib.id_factor(fake, C["ID_F64"], 100, 10, 100, ctypes.byref(g), fake, ws, fake, fake, 10,
                       ctypes.byref(k), ctypes.byref(info), None)
    assert rc == C["ID_ERR_UNSUPPORTED"]
    with pytest.raises(ValueError):
        make_opts(k=3, round_to="f8")


def test_round_flags_pair_with_their_update(lib):
    from paper_2012_00706_amd import C, make_opts
    for prec, rnd in (("mixed_bf16x3", "f32"), ("f64", "f32"), ("mixed_f32", "f16"),
                      ("mixed_bf16", "f16")):
        o = make_opts(k=3, prec=prec, round_to=rnd)
        assert lib.id_workspace_size(10, 10, C["ID_F32"], ctypes.byref(o)) == 0, (prec, rnd)
    for prec, rnd in (("mixed_f32", "f32"), ("mixed_f16", "f16")):
        o = make_opts(k=3, prec=prec, round_to=rnd)
        assert lib.id_workspace_size(10, 10, C["ID_F32"], ctypes.byref(o)) > 0, (prec, rnd)


def _lock_items(shapes, fake):
    from paper_2012_00706_amd import _lib
    items = (_lib.IdBatchItem * len(shapes))()
    for i, (m, n) in enumerate(shapes):
        it = items[i]
        it.A, it.m, it.n, it.lda = fake, m, n, max(m, 1)
        it.work, it.perm, it.R, it.T = fake, fake, fake, fake
        it.ldr = it.ldt = max(min(m, n), 1)
    return items


def test_lockstep_host_checks(lib):
    """id_lockstep_workspace_size / id_factor_lockstep: sizes and argument
    errors before any device call."""
    from paper_2012_00706_amd import C, make_opts
    fake = 0x1000
    o = make_opts(tol=1e-3, prec="mixed_bf16x3")
    items = _lock_items([(300, 150), (2000, 800), (1, 1)], fake)
    ws = lib.id_lockstep_workspace_size(items, 3, C["ID_F32"], ctypes.byref(o))
    assert ws > 0 and ws % 256 == 0
    # more items or larger items need more
    items4 = _lock_items([(300, 150), (2000, 800), (1, 1), (20000, 800)], fake)
    assert lib.id_lockstep_workspace_size(items4, 4, C["ID_F32"], ctypes.byref(o)) > ws
    # invalid: negative batch, a null input, ldr below kcap, an unknown dtype,
    # more than 49152 rows, refused flags
    assert lib.id_lockstep_workspace_size(items, -1, C["ID_F32"], ctypes.byref(o)) == 0
    bad = _lock_items([(300, 150)], fake)
    bad[0].A = None
    assert lib.id_lockstep_workspace_size(bad, 1, C["ID_F32"], ctypes.byref(o)) == 0
    bad = _lock_items([(300, 150)], fake)
    bad[0].ldr = 10
    assert lib.id_lockstep_workspace_size(bad, 1, C["ID_F32"], ctypes.byref(o)) == 0
    assert lib.id_lockstep_workspace_size(items, 3, 7, ctypes.byref(o)) == 0
    tall = _lock_items([(49153, 4)], fake)
    assert lib.id_lockstep_workspace_size(tall, 1, C["ID_F32"], ctypes.byref(o)) == 0
    assert lib.id_factor_lockstep(tall, 1, C["ID_F32"], ctypes.byref(o), fake, 1 << 30,
                                  None) == C["ID_ERR_UNSUPPORTED"]
    ok = _lock_items([(49152, 4)], fake)
    assert lib.id_lockstep_workspace_size(ok, 1, C["ID_F32"], ctypes.byref(o)) > 0
    g = make_opts(tol=1e-3, gram=True)
    assert lib.id_factor_lockstep(items, 3, C["ID_F32"], ctypes.byref(g), fake, ws,
                                  None) == C["ID_ERR_UNSUPPORTED"]
    # workspace too small or missing, and an item without a workspace
    assert lib.id_factor_lockstep(items, 3, C["ID_F32"], ctypes.byref(o), fake, ws - 256,
                                  None) == C["ID_ERR_WORKSPACE"]
    assert lib.id_factor_lockstep(items, 3, C["ID_F32"], ctypes.byref(o), None, ws,
                                  None) == C["ID_ERR_WORKSPACE"]
    nowork = _lock_items([(300, 150)], fake)
    nowork[0].work = None
    assert lib.id_factor_lockstep(nowork, 1, C["ID_F32"], ctypes.byref(o), fake, ws,
                                  None) == C["ID_ERR_WORKSPACE"]
    # an empty batch does nothing
    assert lib.id_factor_lockstep(items, 0, C["ID_F32"], ctypes.byref(o), None, 0,
                                  None) == C["ID_OK"]


def test_cholqr_host_checks(lib):
    """ID_FLAG_CHOLQR: its workspace holds two m x n FP64 copies, and every
    refusal (flag combinations, m < n, short workspace, the entry points that
    do not take it) comes back before any device call."""
    from paper_2012_00706_amd import C, _lib, make_opts
    fake = ctypes.c_void_p(0x1000)
    k = ctypes.c_int64(0)
    info = ctypes.c_int32(0)
    o = make_opts(tol=1e-3, cholqr=True)
    ws = lib.id_workspace_size(1000, 200, C["ID_F32"], ctypes.byref(o))
    assert ws >= 2 * 1000 * 200 * 8 + 7 * 200 * 200 * 8
    assert ws > lib.id_workspace_size(1000, 200, C["ID_F32"], ctypes.byref(make_opts(tol=1e-3)))

    def run(opts, m=1000, n=200, work_bytes=ws):
        return lib.id_factor(fake, C["ID_F32"], m, n, m, ctypes.byref(opts), fake, work_bytes,
                             fake, fake, n, ctypes.byref(k), ctypes.byref(info), None)
    assert run(o, work_bytes=ws - 1) == C["ID_ERR_WORKSPACE"]
    assert run(o, m=100, n=200) == C["ID_ERR_UNSUPPORTED"]  # m < n
    both = make_opts(tol=1e-3, cholqr=True)
    both.flags |= C["ID_FLAG_GRAM"]
    assert lib.id_workspace_size(1000, 200, C["ID_F32"], ctypes.byref(both)) == 0
    assert run(both) == C["ID_ERR_ARG"]
    for extra in ("ID_FLAG_NO_PIVOT", "ID_FLAG_PROFILE"):
        x = make_opts(tol=1e-3, cholqr=True)
        x.flags |= C[extra]
        assert run(x) == C["ID_ERR_UNSUPPORTED"], extra
    r = make_opts(tol=1e-3, prec="mixed_f32", round_to="f32", cholqr=True)
    assert run(r) == C["ID_ERR_UNSUPPORTED"]
    rc = lib.id_factor_noalloc(fake, C["ID_F64"], 100, 10, 100, ctypes.byref(o), fake, fake, 10,
                               ctypes.byref(k), ctypes.byref(info), None)
    assert rc == C["ID_ERR_UNSUPPORTED"]
    items = _lock_items([(300, 40), (200, 30)], fake)
    assert lib.id_factor_lockstep(items, 2, C["ID_F32"], ctypes.byref(o), fake, 1 << 30,
                                  None) == C["ID_ERR_UNSUPPORTED"]
    assert lib.id_status_string(C["ID_INFO_CHOLQR_BREAKDOWN"]).decode() != "unknown code"
