"""Build-level checks of the gfx950 kernels (no GPU): none spills to scratch.

The compiler's kernel-resource remarks are written next to each object by
paper_1111_6900_amd/build.py.  A kernel that spills registers to scratch
memory in its inner loop runs several times slower.  Only the 1-wave
256x256 int8 product kernel, which holds 256 accumulators per lane, is
allowed a few bytes.
"""
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "paper_1111_6900_amd", "_build")
ALLOWED = {"gemm_mfma_kernelILi256ELi256ELi128ELi128E": 64}


def kernel_resources():
    files = glob.glob(os.path.join(BUILD, "*.resources.txt"))
    if not files:
        pytest.skip("library not built here")
    kernels = {}
    for fn in files:
        name = None
        for line in open(fn):
            m = re.search(r"Function Name: (\S+)", line)
            if m:
                name = m.group(1)
                kernels[name] = {}
                continue
            m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[bytes/lane\]| \[bytes/block\]| \[waves/SIMD\])?: (\d+)", line)
            if m and name:
                kernels[name][m.group(1).strip()] = int(m.group(2))
    return kernels


def test_no_kernel_spills():
    kernels = kernel_resources()
    assert len(kernels) > 20
    for name, res in kernels.items():
        limit = next((v for k, v in ALLOWED.items() if k in name), 0)
        assert res.get("ScratchSize", 0) <= limit, (name, res)


def test_product_kernels_fit_lds_and_registers():
    kernels = kernel_resources()
    gemms = {n: r for n, r in kernels.items() if "gemm_" in n}
    assert gemms
    for name, res in gemms.items():
        assert res.get("LDS Size", 0) <= 160 * 1024, name
        assert res.get("VGPRs", 0) <= 256 and res.get("AGPRs", 0) <= 256, name
