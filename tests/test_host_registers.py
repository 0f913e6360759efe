"""Register and scratch budgets of the built gfx950 kernels (host only).

Reads the code object that the build embedded in libcgp.so (the library's
own `.hip_fatbin` section, unbundled with the ROCm LLVM tools) and checks
the budgets the kernels' launch shapes rely on:

* no kernel spills to scratch;
* the one-layer fused stage kernels with a compile-time transform length at
  c = 2 use at most 128 VGPRs per lane, so that two 512-thread blocks share a
  CU (four waves per SIMD).  Ensembles of many blocks need that: at 129-132
  VGPRs the 64-basin FP64 ensemble ran a quarter slower.

Both budgets hold for the measurement build (libcgp_stamps.so) too, so that
its phase stamps time the same launch shapes.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1308_3290_amd", "libcgp.so")
STAMPS_LIB = os.path.join(ROOT, "paper_1308_3290_amd", "libcgp_stamps.so")
TOOLS = "/opt/rocm/llvm/bin"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"


@pytest.fixture(scope="module", params=[LIB, STAMPS_LIB], ids=["libcgp", "libcgp_stamps"])
def kernels(request, tmp_path_factory):
    LIB = request.param
    tools = [os.path.join(TOOLS, t) for t in ("llvm-objcopy", "clang-offload-bundler",
                                              "llvm-readelf")]
    if not os.path.exists(LIB) or not all(os.path.exists(t) for t in tools):
        pytest.skip("built library or ROCm LLVM tools missing")
    objcopy, bundler, readelf = tools
    d = tmp_path_factory.mktemp("codeobj")
    fat, lib_copy = d / "fatbin", d / "lib.so"
    subprocess.run([objcopy, f"--dump-section=.hip_fatbin={fat}", LIB, str(lib_copy)],
                   check=True, capture_output=True)
    # the section holds one offload bundle per object file, back to back
    data = fat.read_bytes()
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    starts = [m.start() for m in re.finditer(re.escape(magic), data)]
    notes = ""
    for n, (a, b) in enumerate(zip(starts, starts[1:] + [len(data)])):
        part, co = d / f"bundle{n}", d / f"code{n}.hsaco"
        part.write_bytes(data[a:b])
        subprocess.run([bundler, "--unbundle", "--type=o", f"--input={part}",
                        f"--targets={TARGET}", f"--output={co}"], check=True, capture_output=True)
        notes += subprocess.run([readelf, "--notes", str(co)], check=True, capture_output=True,
                                text=True).stdout
    meta, cur = {}, None
    # within a kernel's map the keys are sorted: its .name follows its
    # arguments' names and precedes the register counts
    for line in notes.splitlines():
        m = re.match(r"\s+\.name:\s+(\S+)", line)
        if m:
            cur = m.group(1)
            continue
        m = re.match(r"\s+\.(vgpr_count|private_segment_fixed_size):\s+(\d+)", line)
        if m and cur and cur.startswith("_ZN3cgp"):
            meta.setdefault(cur, {})[m.group(1)] = int(m.group(2))
    assert meta, "no kernel metadata found"
    return meta


def test_no_kernel_uses_scratch(kernels):
    spill = {k: v["private_segment_fixed_size"] for k, v in kernels.items()
             if v.get("private_segment_fixed_size", 0) > 0}
    assert not spill, spill


def test_fused_c2_kernels_fit_two_blocks_per_cu(kernels):
    # k_prolong_stencil<T, C = 2, TJ = 2, LC, NEXT = true, NTS>, LC = 128 .. 512,
    # with and without the write-through stores of the new vorticity
    pat = re.compile(r"_ZN3cgp17k_prolong_stencilI([df])Li2ELi2ELi(\d+)ELb1ELb[01]E")
    seen = 0
    for name, v in kernels.items():
        m = pat.match(name)
        if m and m.group(2) != "0":
            seen += 1
            assert v["vgpr_count"] <= 128, (name, v)
    assert seen == 16  # two element types x four compile-time lengths x two store forms


def test_metadata_covers_every_translation_unit(kernels):
    names = " ".join(kernels)
    for k in ("k_col_solve", "k_prolong_stencilI", "k_prolong_stencil2", "k_adjoint_fused",
              "k_stencil_rk3", "k_mg_smooth", "k_diag_partial"):
        assert k in names, k
