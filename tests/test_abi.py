"""The C-ABI library loads, exports every symbol include/fdk.h declares, and
rejects invalid arguments before touching the GPU (no compute calls here)."""
import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import paper_1104_5243_amd as fdk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdk.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fdk_\w+)\s*\(", text)))


def test_header_declares_what_the_binding_lists():
    assert declared_symbols() == sorted(fdk.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = fdk.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_conv_flag_constants_match_header():
    text = open(HEADER).read()
    defs = dict(re.findall(r"#define FDK_CONV_(\w+) (\d+)", text))
    assert defs and {k: int(v) for k, v in defs.items()} == {
        k: getattr(fdk, "CONV_" + k) for k in defs}


@pytest.mark.parametrize("extra", [1, 2])
def test_conv_relu_mask_excludes_relu_and_accumulate(extra):
    rc = fdk.lib().fdk_conv_rows(FAKE, FAKE, FAKE, None, 4, 16, 32, 32, 9, 4,
                                 fdk.CONV_RELU_MASK | extra, None)
    assert rc == fdk.FDK_ERR_INVALID_ARG
    assert "RELU_MASK" in fdk.last_error()


def test_version():
    assert fdk.version() >> 16 == 1


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


def _call(**over):
    P = np.tile(np.eye(3, 4), (2, 1, 1)).astype(np.float64)
    o = (ctypes.c_float * 3)(0.0, 0.0, 0.0)
    args = dict(volume=FAKE, N=8, vs=1.0, origin=o, proj=FAKE, dtype=0, n_views=2, H=4, W=4,
                P=P.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), scale=None, flags=0)
    args.update(over)
    rc = fdk.lib().fdk_backproject_ex(args["volume"], args["N"], args["vs"], args["origin"],
                                      args["proj"], args["dtype"], args["n_views"], args["H"],
                                      args["W"], args["P"], args["scale"], args["flags"], None)
    return rc, fdk.last_error()


@pytest.mark.parametrize("over,needle", [
    (dict(volume=None), "volume"),
    (dict(N=0), "N=0"),
    (dict(N=5000), "N=5000"),
    (dict(vs=0.0), "voxel_size"),
    (dict(vs=float("nan")), "voxel_size"),
    (dict(origin=None), "origin"),
    (dict(n_views=-1), "n_views"),
    (dict(H=0), "detector"),
    (dict(W=40000), "detector"),
    (dict(proj=None), "proj_stack"),
    (dict(P=None), "P_mats"),
    (dict(dtype=7), "proj_dtype"),
    (dict(flags=9), "flags"),
])
def test_invalid_arguments_are_rejected(over, needle):
    rc, msg = _call(**over)
    assert rc == fdk.FDK_ERR_INVALID_ARG
    assert needle in msg


def test_nonfinite_matrix_rejected():
    P = np.tile(np.eye(3, 4), (2, 1, 1)).astype(np.float64)
    P[1, 2, 3] = np.inf
    rc, msg = _call(P=P.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == fdk.FDK_ERR_INVALID_ARG and "P_mats[23]" in msg


def test_bad_view_scale_rejected():
    s = (ctypes.c_float * 2)(1.0, -4.0)
    rc, msg = _call(scale=s)
    assert rc == fdk.FDK_ERR_INVALID_ARG and "view_scale[1]" in msg


def test_plain_kernel_rejects_reduced_precision():
    rc, msg = _call(dtype=1, flags=1)
    assert rc == fdk.FDK_ERR_UNSUPPORTED


def test_zero_views_is_a_noop_without_pointers():
    rc, _ = _call(n_views=0, proj=None, P=None)
    assert rc == fdk.FDK_OK


def test_batch_setting():
    L = fdk.lib()
    old = L.fdk_set_batch(0)
    assert 1 <= old <= 1024
    assert L.fdk_set_batch(1025) == fdk.FDK_ERR_INVALID_ARG
    assert L.fdk_set_batch(-1) == fdk.FDK_ERR_INVALID_ARG
    assert L.fdk_set_batch(496) == 496
    assert L.fdk_set_batch(7) == 7
    assert L.fdk_set_batch(old) == old


def test_layout_setting():
    L = fdk.lib()
    old = L.fdk_set_layout(-1)
    assert 0 <= old <= 4
    assert L.fdk_set_layout(5) == fdk.FDK_ERR_INVALID_ARG
    assert L.fdk_set_layout(-2) == fdk.FDK_ERR_INVALID_ARG
    for name, code in fdk.LAYOUTS.items():
        assert fdk.set_layout(name) == name
        assert L.fdk_set_layout(-1) == code
    assert L.fdk_set_layout(old) == old


def test_row_clamp_setting():
    L = fdk.lib()
    old = L.fdk_set_row_clamp(-1)
    assert old in (0, 1)
    assert L.fdk_set_row_clamp(2) == fdk.FDK_ERR_INVALID_ARG
    assert L.fdk_set_row_clamp(-2) == fdk.FDK_ERR_INVALID_ARG
    assert fdk.set_row_clamp(True) is True
    assert L.fdk_set_row_clamp(-1) == 1
    assert fdk.set_row_clamp(False) is False
    assert fdk.set_row_clamp(None) is False
    assert L.fdk_set_row_clamp(old) == old


C_PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "fdk.h"

int main(void)
{
    float origin[3] = {0.0f, 0.0f, 0.0f};
    double P[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
    int rc;
    if ((fdk_version() >> 16) != 1) return 1;
    /* rejected before any GPU work: no volume */
    rc = fdk_backproject(NULL, 8, 1.0f, origin, NULL, 1, 4, 4, P, NULL);
    if (rc != FDK_ERR_INVALID_ARG || strstr(fdk_last_error(), "volume") == NULL) return 2;
    /* zero views: a no-op */
    if (fdk_backproject((float*)16, 8, 1.0f, origin, NULL, 0, 4, 4, NULL, NULL) != FDK_OK) return 3;
    if (fdk_conv_rows_wgrad_workspace(32, 32, 9) == 0) return 4;
    printf("ok\n");
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_header_is_c_and_library_links_from_c(tmp_path):
    """include/fdk.h compiles as C99 (no C++ in the ABI) and a C program
    linked against libfdk.so runs the entry points that need no GPU."""
    fdk.lib()
    src = tmp_path / "use_fdk.c"
    src.write_text(C_PROGRAM)
    exe = tmp_path / "use_fdk"
    lib_dir = os.path.dirname(fdk.LIB_PATH)
    cmd = ["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
           "-o", str(exe), "-L", lib_dir, "-l:" + os.path.basename(fdk.LIB_PATH),
           "-Wl,-rpath," + lib_dir]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, (out.returncode, out.stdout, out.stderr)
    assert out.stdout.strip() == "ok"


def test_noalloc_rejects_a_view_larger_than_its_scratch():
    """A single staged view beyond the fixed scratch array is refused before
    any HIP call (8192 x 8192 FP32 in the default layout: ~541 MB)."""
    P = np.tile(np.eye(3, 4), (2, 1, 1)).astype(np.float64)
    o = (ctypes.c_float * 3)(0.0, 0.0, 0.0)
    rc = fdk.lib().fdk_backproject_noalloc(FAKE, 8, 1.0, o, FAKE, 0, 2, 8192, 8192,
                                           P.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           None, None)
    assert rc == fdk.FDK_ERR_UNSUPPORTED
    assert "scratch" in fdk.last_error()


@pytest.mark.parametrize("over,needle", [(dict(volume=None), "volume"), (dict(dtype=5), "proj_dtype"),
                                         (dict(scale=-1.0), "view_scale")])
def test_noalloc_validates_before_launch(over, needle):
    P = np.tile(np.eye(3, 4), (2, 1, 1)).astype(np.float64)
    o = (ctypes.c_float * 3)(0.0, 0.0, 0.0)
    a = dict(volume=FAKE, dtype=0, scale=None)
    a.update(over)
    sc = None
    if a["scale"] is not None:
        sc = (ctypes.c_float * 2)(a["scale"], 1.0)
    rc = fdk.lib().fdk_backproject_noalloc(a["volume"], 8, 1.0, o, FAKE, a["dtype"], 2, 4, 4,
                                           P.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           sc, None)
    assert rc == fdk.FDK_ERR_INVALID_ARG
    assert needle in fdk.last_error()
