"""Register and scratch footprint of the sweep kernels as compiled into libnfm.so (CPU: the code
objects' metadata is read from the built library, nothing runs on a GPU).

The launch design rests on these numbers: the SIMD-exclusive queue form must hold more than half
of a SIMD's 512 registers (so no other wave is placed beside it), the queue form for L <= 8 at
most 168 VGPRs (three waves per SIMD), and no sweep kernel may spill registers to scratch memory
(a spill on the decision chain would cost far more than any of the forms' differences)."""
import os
import re
import shutil
import subprocess

import pytest
import yaml

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2011_08560_amd", "libnfm.so")
TOOLS = "/opt/rocm/llvm/bin"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"


def _tool(name):
    p = os.path.join(TOOLS, name)
    return p if os.path.exists(p) else shutil.which(name)


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    tools = [_tool(t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf")]
    if not os.path.exists(LIB) or not all(tools):
        pytest.skip("library or LLVM tools not available")
    objcopy, bundler, readelf = tools
    d = tmp_path_factory.mktemp("co")
    fat = d / "fatbin"
    subprocess.run([objcopy, "--dump-section", f".hip_fatbin={fat}", LIB, str(d / "copy.so")], check=True,
                   capture_output=True)
    data = fat.read_bytes()
    starts = [m.start() for m in re.finditer(re.escape(b"__CLANG_OFFLOAD_BUNDLE__"), data)]
    out = {}
    for i, s in enumerate(starts):
        part = d / f"b{i}"
        part.write_bytes(data[s:starts[i + 1] if i + 1 < len(starts) else len(data)])
        co = d / f"b{i}.co"
        r = subprocess.run([bundler, "--unbundle", "--type=o", "--input", str(part), f"--targets={TARGET}",
                            "--output", str(co)], capture_output=True, text=True)
        if r.returncode != 0:
            continue
        notes = subprocess.run([readelf, "--notes", str(co)], capture_output=True, text=True, check=True).stdout
        m = re.search(r"^\s*---\n(.*?)^\s*\.\.\.\s*$", notes, re.S | re.M)
        if not m:
            continue
        meta = yaml.safe_load("---\n" + m.group(1))
        for k in meta.get("amdhsa.kernels", []):
            out[k[".name"]] = k
    assert out, "no kernel metadata found in the library"
    return out


def _find(kernels, pattern):
    hits = {n: k for n, k in kernels.items() if re.search(pattern, n)}
    assert hits, pattern
    return hits


def test_simd_exclusive_form_claims_the_simd(kernels):
    # k_sweeps_queue<SPEC, 12, true>: mangled ...k_sweeps_queueILb{0,1}ELi12ELb1E...
    for name, k in _find(kernels, r"k_sweeps_queueILb[01]ELi12ELb1E").items():
        assert k[".agpr_count"] == 256, name
        assert k[".vgpr_count"] + k[".agpr_count"] > 256, name       # two of them do not fit in 512


def test_small_lattice_queue_form_keeps_three_waves(kernels):
    for name, k in _find(kernels, r"k_sweeps_queueILb0ELi8ELb0E").items():
        assert k[".vgpr_count"] <= 168 and k[".agpr_count"] == 0, (name, k[".vgpr_count"])


def test_sweep_kernels_do_not_spill(kernels):
    sweeps = _find(kernels, r"k_sweeps")
    assert len(sweeps) >= 30
    for name, k in sweeps.items():
        assert k.get(".vgpr_spill_count", 0) == 0, name
        assert k.get(".private_segment_fixed_size", 0) == 0, name
