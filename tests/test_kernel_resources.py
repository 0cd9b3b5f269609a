"""CPU: no kernel of the built library uses scratch memory or spills VGPRs to it.

Private (scratch) memory in these kernels has come from local arrays indexed
at run time; every lane then writes them to memory, which once cost the batch
box sum several times its useful HBM writes. The check reads the kernel
descriptors of the gfx950 code object embedded in libhpf.so (built here from
source) with the ROCm LLVM tools; it needs no GPU. (SGPR spills go to VGPR
lanes, not to memory, and are not checked.)
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1310_2041_amd", "libhpf.so")
LLVM = "/opt/rocm/llvm/bin"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"


def _tool(name):
    p = os.path.join(LLVM, name)
    return p if os.path.exists(p) else shutil.which(name)


def kernel_metadata(tmp_path):
    """{kernel symbol: {field: int}} from the code object's metadata note."""
    objcopy, bundler, readelf = (_tool(t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf"))
    if not (objcopy and bundler and readelf):
        pytest.skip("ROCm LLVM tools not found")
    if not os.path.exists(LIB):
        pytest.skip("libhpf.so not built")
    fat, co = str(tmp_path / "fat.bin"), str(tmp_path / "dev.co")
    subprocess.run([objcopy, "--dump-section", f".hip_fatbin={fat}", LIB, str(tmp_path / "copy.so")],
                   check=True, capture_output=True)
    subprocess.run([bundler, "--unbundle", "--type=o", f"--targets={TARGET}", f"--input={fat}",
                    f"--output={co}"], check=True, capture_output=True)
    notes = subprocess.run([readelf, "--notes", co], check=True, capture_output=True, text=True).stdout
    out, cur = {}, None
    for line in notes.splitlines():
        m = re.match(r"\s*\.name:\s+(\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.match(r"\s*\.(private_segment_fixed_size|vgpr_spill_count|sgpr_spill_count|vgpr_count):\s+(\d+)",
                     line)
        if m and cur is not None:
            cur[m.group(1)] = int(m.group(2))
    return out


def test_no_kernel_uses_scratch_or_spills(tmp_path):
    md = kernel_metadata(tmp_path)
    kernels = {k: v for k, v in md.items() if k.startswith("_ZN3hpf")}
    assert len(kernels) > 30, "kernel metadata not found"
    bad = {k: v for k, v in kernels.items()
           if v.get("private_segment_fixed_size", 0) or v.get("vgpr_spill_count", 0)}
    assert not bad, bad


def test_fused_pass_register_budget(tmp_path):
    """The production fused advance + deposit kernel (512 threads, r0 = 0, no thermostat)
    keeps 4 waves per SIMD (at most 128 VGPRs of 512), so that two workgroups share a CU;
    every other single-system variant (r0 != 0, the Andersen thermostat, 768-thread
    workgroups) keeps at least 3 (at most 168). The batched passes keep 4 without the
    thermostat and 3 with it."""
    md = kernel_metadata(tmp_path)
    fused = {k: v for k, v in md.items() if "advance_scatter" in k}
    assert len(fused) >= 16
    for k, v in fused.items():
        single = re.search(r"k_advance_scatterILb([01])ELi(\d+)ELb([01])ELb([01])E", k)
        if single:
            r0z, threads, thermo = single.group(1) == "1", int(single.group(2)), single.group(4) == "1"
            limit = 128 if (threads == 512 and r0z and not thermo) else 168
        else:
            thermo = re.search(r"Lb([01])EEEv", k).group(1) == "1"
            limit = 168 if thermo else 128
        assert v["vgpr_count"] <= limit, (k, v)
