"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/recon.h, and validates parameters on the host."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "recon.h")


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:recon_status|void|const char\s*\*)\s*\*?\s*(recon_\w+)\s*\(",
                                 text, flags=re.M)))


@pytest.fixture(scope="module")
def recon():
    from paper_1910_08498_amd import recon as r
    if not os.path.exists(r.LIB_PATH):
        pytest.fail("librecon.so is not built (run __graft_entry__.build())")
    r.load_library()
    return r


def test_header_declares_the_boundary():
    names = header_functions()
    for must in ("recon_init", "recon_insert_batch", "recon_finalize", "recon_query_sizes",
                 "recon_destroy", "recon_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(recon):
    lib = ctypes.CDLL(recon.LIB_PATH)
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_default_params_and_sizes(recon):
    p = recon.recon_default_params(128)
    assert p.n == 128 and p.max_batch == 1500 and p.table_size == 10000
    assert abs(p.blob_radius - 1.9) < 1e-6 and p.blob_alpha == 15.0 and p.r_max == 64.0
    g, w, ws = recon.recon_query_sizes(p)
    assert g == 129 ** 3 * 8 and w == 129 ** 3 * 4
    # table + orientations + plan at least
    assert ws >= 10000 * 8 + 1500 * 64
    p.max_batch = 3000
    assert recon.recon_query_sizes(p)[2] > ws


def test_degenerate_blob_rejected(recon):
    # alpha = 0 with order m > 0: the normaliser I_m(0) is zero
    p = recon.recon_default_params(128)
    p.blob_alpha, p.blob_order = 0.0, 2
    with pytest.raises(recon.ReconError) as ei:
        recon.recon_query_sizes(p)
    assert ei.value.status == recon.RECON_EINVAL
    p.blob_order = 0                            # alpha = 0, m = 0: the box profile b = 1
    recon.recon_query_sizes(p)


def test_on_the_fly_weights_need_no_table(recon):
    p = recon.recon_default_params(128)
    _, _, ws_table = recon.recon_query_sizes(p)
    p.table_size = 0                            # weights evaluated on the fly
    _, _, ws_otf = recon.recon_query_sizes(p)
    assert ws_otf < ws_table
    p.blob_alpha, p.blob_order = 60.0, 8        # the steepest accepted blob still converges
    recon.recon_query_sizes(p)


@pytest.mark.parametrize("field,value", [
    ("n", 63), ("n", 2), ("n", 2048), ("blob_radius", 0.0), ("blob_radius", 0.99), ("blob_radius", 3.5),
    ("blob_alpha", -1.0), ("blob_order", 9), ("table_size", 1), ("table_lerp", 2),
    ("r_max", 64.5), ("r_max", 0.0), ("max_batch", 0), ("slice_dtype", 7), ("slice_dtype", -1),
])
def test_invalid_params_rejected(recon, field, value):
    p = recon.recon_default_params(128)
    setattr(p, field, value)
    with pytest.raises(recon.ReconError) as ei:
        recon.recon_query_sizes(p)
    assert ei.value.status == recon.RECON_EINVAL
    assert recon.load_library().recon_last_error().decode() != ""


def test_null_arguments_rejected(recon):
    lib = recon.load_library()
    assert lib.recon_default_params(64, None) == recon.RECON_EINVAL
    assert lib.recon_query_sizes(None, None, None, None) == recon.RECON_EINVAL
    assert lib.recon_insert_batch(None, None, None, None, 0) == recon.RECON_EINVAL
    assert lib.recon_finalize(None, None, ctypes.c_float(0.0)) == recon.RECON_EINVAL
    assert lib.recon_stats(None, None, None) == recon.RECON_EINVAL
    lib.recon_destroy(None)   # ignored


def test_init_rejects_small_workspace_without_touching_device(recon):
    p = recon.recon_default_params(16)
    lib = recon.load_library()
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: rejected before any device call
    rc = lib.recon_init(ctypes.byref(p), fake, fake, fake, 16, None, ctypes.byref(ctx))
    assert rc == recon.RECON_ENOMEM
    assert not ctx.value


def test_version(recon):
    assert "gfx950" in recon.recon_version()


def test_struct_layouts_match_the_header(recon, tmp_path):
    # sizes and offsets from a C program built against include/recon.h
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "recon.h"
int main(void) {
    printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(recon_params), sizeof(recon_config),
           offsetof(recon_config, cu_count), sizeof(recon_tune_opts), offsetof(recon_tune_opts, order_count),
           offsetof(recon_tune_opts, order), sizeof(recon_tune_info));
    return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    want = [ctypes.sizeof(recon.recon_params), ctypes.sizeof(recon.recon_config), recon.recon_config.cu_count.offset,
            ctypes.sizeof(recon.recon_tune_opts), recon.recon_tune_opts.order_count.offset,
            recon.recon_tune_opts.order.offset, ctypes.sizeof(recon.recon_tune_info)]
    assert got == want


def test_static_workspace_rejects_oversized_parameters_before_any_device_call(recon):
    # 2^24 slices per call need ~2.9 GB of orientation records, beyond the
    # static workspace; the size check precedes every device call, so it
    # answers here without a GPU
    p = recon.recon_default_params(128)
    p.max_batch = 1 << 24
    assert recon.recon_query_sizes(p)[2] > (192 << 20)
    lib = recon.load_library()
    ctx = ctypes.c_void_p()
    rc = lib.recon_init_static(ctypes.byref(p), None, None, None, ctypes.byref(ctx))
    assert rc == recon.RECON_ENOMEM and not ctx.value
    assert "static workspace" in lib.recon_last_error().decode()
    # the library's defaults fit every box up to n = 1024
    for n in (64, 128, 256, 512, 1024):
        assert recon.recon_query_sizes(recon.recon_default_params(n))[2] <= (192 << 20)
