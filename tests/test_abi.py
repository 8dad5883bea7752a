"""C-ABI checks that need no GPU: the library loads, exports every function
include/bfx.h declares, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bfx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bfx_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    from paper_1904_06376_amd import _lib
    names = _declared()
    assert len(names) >= 10
    missing = [n for n in names if getattr(_lib.lib, n, None) is None]
    assert not missing, missing
    assert set(names) <= set(_lib.SIGNATURES), set(names) - set(_lib.SIGNATURES)


def test_version_and_error_string():
    from paper_1904_06376_amd import _lib
    assert _lib.lib.bfx_version() >= 10000
    assert isinstance(_lib.lib.bfx_last_error_string(), bytes)


def test_argument_errors_before_device_use():
    from paper_1904_06376_amd._lib import lib
    v = ctypes.c_void_p(16)
    assert lib.bfx_gemm(5, 4, 4, 4, 1.0, v, 4, v, 4, 0.0, v, 4, None, 0, None) == -1
    assert lib.bfx_gemm(6, -1, 4, 4, 1.0, v, 4, v, 4, 0.0, v, 4, None, 0, None) == -2
    assert lib.bfx_gemm(6, 4, 4, 4, 1.0, None, 4, v, 4, 0.0, v, 4, None, 0, None) == -6
    assert lib.bfx_gemm(6, 4, 4, 4, 1.0, v, 3, v, 4, 0.0, v, 4, None, 0, None) == -7
    assert lib.bfx_gemm(6, 4, 4, 4, 1.0, v, 4, v, 4, 0.0, v, 2, None, 0, None) == -12
    assert lib.bfx_gemm(6, 0, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, None, 0, None) == 0
    assert lib.bfx_sgemm_fp32(4, 4, -2, 1.0, v, 4, v, 4, 0.0, v, 4, None, 0, None) == -3
    assert lib.bfx_split_f32(v, -1, 3, v, v, v, None) == -2
    assert lib.bfx_split_f32(v, 8, 4, v, v, v, None) == -3
    assert lib.bfx_split_f32(v, 8, 3, v, v, None, None) == -6
    assert lib.bfx_split_f32(None, 0, 3, None, None, None, None) == 0
    assert lib.bfx_gemm_ws_size(6, 64, 64, 1 << 20) > 0
    assert lib.bfx_gemm_ws_size(6, 512, 512, 256) == 0
    # pre-split planes: P BF16 planes of A and B, M and N padded to 128, K to 32
    assert lib.bfx_gemm_ws_size(6, 4096, 4096, 4096) == 3 * (4096 + 4096) * 4096 * 2
    assert lib.bfx_gemm_ws_size(3, 4000, 4100, 1000) == 2 * (4096 + 4224) * 1024 * 2
    # pre-split block layout: nterms planes of ceil(R/128) x ceil(K/32) blocks of 4096 BF16
    assert lib.bfx_split_blocks_size(3, 200, 77) == 3 * 2 * 3 * 4096 * 2
    assert lib.bfx_split_blocks_size(1, 128, 32) == 4096 * 2
    assert lib.bfx_split_blocks_size(4, 128, 32) == 0
    assert lib.bfx_split_blocks_size(2, 0, 32) == 0
    big = ctypes.c_size_t(1 << 40)
    assert lib.bfx_split_blocks(0, 0, 8, 8, v, 8, v, big, None) == -1
    assert lib.bfx_split_blocks(3, 2, 8, 8, v, 8, v, big, None) == -2
    assert lib.bfx_split_blocks(3, 0, -1, 8, v, 8, v, big, None) == -3
    assert lib.bfx_split_blocks(3, 0, 8, -1, v, 8, v, big, None) == -4
    assert lib.bfx_split_blocks(3, 0, 8, 8, None, 8, v, big, None) == -5
    assert lib.bfx_split_blocks(3, 0, 8, 8, v, 7, v, big, None) == -6
    assert lib.bfx_split_blocks(3, 1, 8, 4, v, 7, v, big, None) == -6
    assert lib.bfx_split_blocks(3, 0, 8, 8, v, 8, None, big, None) == -7
    assert lib.bfx_split_blocks(3, 0, 8, 8, v, 8, ctypes.c_void_p(24), big, None) == -7
    assert lib.bfx_split_blocks(3, 0, 8, 8, v, 8, v, 3 * 4096 * 2 - 1, None) == -8
    assert lib.bfx_split_blocks(3, 0, 0, 8, None, 8, None, 0, None) == 0
    assert lib.bfx_gemm_blocks(2, 4, 4, 4, 1.0, v, v, 0.0, v, 4, None) == -1
    assert lib.bfx_gemm_blocks(6, -1, 4, 4, 1.0, v, v, 0.0, v, 4, None) == -2
    assert lib.bfx_gemm_blocks(6, 4, -1, 4, 1.0, v, v, 0.0, v, 4, None) == -3
    assert lib.bfx_gemm_blocks(6, 4, 4, -1, 1.0, v, v, 0.0, v, 4, None) == -4
    assert lib.bfx_gemm_blocks(6, 4, 4, 4, 1.0, None, v, 0.0, v, 4, None) == -6
    assert lib.bfx_gemm_blocks(6, 4, 4, 4, 1.0, v, ctypes.c_void_p(40), 0.0, v, 4, None) == -7
    assert lib.bfx_gemm_blocks(6, 4, 4, 4, 1.0, v, v, 0.0, None, 4, None) == -9
    assert lib.bfx_gemm_blocks(6, 4, 4, 4, 1.0, v, v, 0.0, v, 3, None) == -10
    assert lib.bfx_gemm_blocks(6, 0, 4, 4, 1.0, None, None, 0.0, None, 4, None) == 0


def test_noalloc_argument_errors_before_device_use():
    from paper_1904_06376_amd._lib import lib
    v = ctypes.c_void_p(16)
    assert lib.bfx_gemm_noalloc_scratch_bytes() == 64 << 20
    assert lib.bfx_gemm_noalloc(5, 4, 4, 4, 1.0, v, 4, v, 4, 0.0, v, 4, None) == -1
    assert lib.bfx_gemm_noalloc(6, 4, -1, 4, 1.0, v, 4, v, 4, 0.0, v, 4, None) == -3
    assert lib.bfx_gemm_noalloc(6, 4, 4, 4, 1.0, v, 4, None, 4, 0.0, v, 4, None) == -8
    assert lib.bfx_gemm_noalloc(6, 4, 4, 4, 1.0, v, 4, v, 4, 0.0, None, 4, None) == -11
    assert lib.bfx_gemm_noalloc(6, 0, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, None) == 0
