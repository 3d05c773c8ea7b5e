"""C ABI: the library is built, loads, exports every declared entry point, and
validates arguments on its host-only paths (no GPU needed)."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    hdr = open(os.path.join(ROOT, "include", "gcp.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(gcp_[a-z_]+)\s*\(", hdr)))


@pytest.fixture(scope="module")
def lib():
    import paper_1512_07236_amd as gcp
    if not os.path.exists(gcp.LIB_PATH):
        pytest.fail("libgcp.so is not built (run __graft_entry__.build())")
    return gcp.load_library()


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("gcp_create", "gcp_init", "gcp_purify", "gcp_backward", "gcp_destroy",
              "gcp_get_history", "gcp_last_error", "gcp_options_default"):
        assert s in syms


def test_every_declared_symbol_is_exported(lib):
    for s in declared_symbols():
        assert hasattr(lib, s), s


def test_struct_layout_matches_c_compiler(tmp_path):
    """The ctypes mirrors of gcp_options / gcp_result have the C layout."""
    import subprocess
    import paper_1512_07236_amd as gcp
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "gcp.h"\n'
        'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(gcp_options),'
        ' sizeof(gcp_verify_result), offsetof(gcp_verify_result, ms),'
        ' sizeof(gcp_result), offsetof(gcp_options, fold_every),'
        ' offsetof(gcp_options, checkpoint_every), offsetof(gcp_result, gemm_launches),'
        ' offsetof(gcp_result, mfma_flops), offsetof(gcp_options, floor_ddbar),'
        ' offsetof(gcp_result, host_syncs), offsetof(gcp_options, ksplit),'
        ' offsetof(gcp_options, final_ddbar), offsetof(gcp_options, final_precision));return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert got == [ctypes.sizeof(gcp.Options), ctypes.sizeof(gcp.CVerify), gcp.CVerify.ms.offset,
                   ctypes.sizeof(gcp.CResult),
                   gcp.Options.fold_every.offset, gcp.Options.checkpoint_every.offset,
                   gcp.CResult.gemm_launches.offset, gcp.CResult.mfma_flops.offset,
                   gcp.Options.floor_ddbar.offset, gcp.CResult.host_syncs.offset,
                   gcp.Options.ksplit.offset, gcp.Options.final_ddbar.offset,
                   gcp.Options.final_precision.offset]


def test_options_default(lib):
    import paper_1512_07236_amd as gcp
    o = gcp.default_options()
    assert (o.precision, o.max_iter, o.tol_ddbar, o.tol_idem, o.fold_every, o.profile,
            o.keep_iterates, o.bwd_precision, o.late_precision, o.switch_ddbar, o.method,
            o.init_mode, o.alpha, o.delta, o.hole, o.checkpoint_every, o.sync_every, o.ksplit) == \
        (0, 100, 1e-6, 0.0, 0, 0, 0, 0, -1, 0.0, 0, 0, 0.5, 2.0 / 3.0, 0, 0, 4, 0)
    assert math.isnan(o.floor_ddbar)
    assert (o.final_precision, o.final_ddbar) == (-1, 0.0)
    assert lib.gcp_options_default(None) == gcp.ERR_INVALID_ARG


def test_create_rejects_bad_arguments_before_touching_the_device(lib):
    import paper_1512_07236_amd as gcp
    h = ctypes.c_void_p()
    assert lib.gcp_create(None, 16, None, None) == gcp.ERR_INVALID_ARG
    assert lib.gcp_create(ctypes.byref(h), 0, None, None) == gcp.ERR_INVALID_ARG
    assert b"M must be" in lib.gcp_last_error(None)
    o = gcp.default_options()
    o.precision = 99
    assert lib.gcp_create(ctypes.byref(h), 16, ctypes.byref(o), None) == gcp.ERR_INVALID_ARG
    o = gcp.default_options()
    o.tol_ddbar = -1.0
    assert lib.gcp_create(ctypes.byref(h), 16, ctypes.byref(o), None) == gcp.ERR_INVALID_ARG
    for field, bad in (("keep_iterates", 2), ("bwd_precision", int(gcp.Precision.BF16))):
        o = gcp.default_options()
        setattr(o, field, bad)
        assert lib.gcp_create(ctypes.byref(h), 16, ctypes.byref(o), None) == gcp.ERR_INVALID_ARG
        assert b"bwd_precision" in lib.gcp_last_error(None)
    for field, bad in (("method", 2), ("init_mode", 3), ("alpha", 1.5), ("delta", 0.4),
                       ("hole", 2), ("checkpoint_every", -1)):
        o = gcp.default_options()
        setattr(o, field, bad)
        assert lib.gcp_create(ctypes.byref(h), 16, ctypes.byref(o), None) == gcp.ERR_INVALID_ARG
        assert b"init_mode" in lib.gcp_last_error(None)
    for field, bad in (("late_precision", 7), ("late_precision", -2), ("switch_ddbar", -1.0),
                       ("final_precision", 7), ("final_ddbar", -1.0)):
        o = gcp.default_options()
        setattr(o, field, bad)
        assert lib.gcp_create(ctypes.byref(h), 16, ctypes.byref(o), None) == gcp.ERR_INVALID_ARG
        assert b"late_precision" in lib.gcp_last_error(None)
    # the final phase's threshold lies below the late phase's
    o = gcp.default_options()
    o.late_precision, o.switch_ddbar = int(gcp.Precision.FP16X3), 1e-3
    o.final_precision, o.final_ddbar = int(gcp.Precision.FP64), 1e-2
    assert lib.gcp_create(ctypes.byref(h), 16, ctypes.byref(o), None) == gcp.ERR_INVALID_ARG
    for field, bad in (("sync_every", 0), ("floor_ddbar", -1.0), ("ksplit", -1), ("ksplit", 65)):
        o = gcp.default_options()
        setattr(o, field, bad)
        assert lib.gcp_create(ctypes.byref(h), 16, ctypes.byref(o), None) == gcp.ERR_INVALID_ARG
        assert b"sync_every" in lib.gcp_last_error(None)
    assert h.value is None
    # NULL contexts are rejected, not dereferenced
    assert lib.gcp_init(None, None, 16, 1, 0.0, 1.0) == gcp.ERR_INVALID_ARG
    assert lib.gcp_purify(None, None, 0, 16, None) == gcp.ERR_INVALID_ARG
    assert lib.gcp_backward(None, None, 16, None, 16, 0, None) == gcp.ERR_INVALID_ARG
    assert lib.gcp_verify(None, None, 0, 16, None, 16, None) == gcp.ERR_INVALID_ARG
    n = ctypes.c_int32()
    assert lib.gcp_get_history(None, None, 0, ctypes.byref(n)) == gcp.ERR_INVALID_ARG
    lib.gcp_destroy(None)


def test_precision_names():
    import paper_1512_07236_amd as gcp
    assert gcp.Precision.parse("fp16x3") == gcp.Precision.FP16X3
    assert gcp.PRODUCTS[gcp.Precision.BF16X6] == 6
