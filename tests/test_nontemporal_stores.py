"""Every global store of every step kernel is a nontemporal (streaming) store.

The step kernels write each population once and never read it back within the step, so
their stores carry the nontemporal hint (`nt`), which keeps them from allocating in the
caches.  The hint is a performance property that tests of the results cannot see, and
compiler transformations can drop it (a restructured loop once lost it on the FP32 A-B
kernel's LDS path, 8 % slower): this test compiles the step-kernel sources for gfx950 to
assembly (host-side cross compilation, no GPU) and checks each `global_store` in the
functions named k_step*.

One deliberate exception: the D3Q19 AA odd step through LDS with 16- or 32-bit storage
writes its ten directions with c_x != 0 (runs shifted by one element, each 64-element run
shared by two wavefronts) without the hint, so exactly ten of its stores are plain.

Loads keep the default policy except in the AA even steps, whose own-slot reads carry the
hint where it measured faster: all 19 in the D3Q19 step, all 9 in the D2Q9 step with FP64
storage (checked the same way).
"""
import functools
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2108_13241_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@functools.lru_cache(maxsize=None)
def _device_asm(src):
    """gfx950 assembly of one kernel source, compiled once per test session."""
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "k.s")
        subprocess.run([HIPCC, "-O3", "-std=c++17", "-ffp-contract=on", "--offload-arch=gfx950",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-x", "hip",
                        "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out],
                       check=True, capture_output=True)
        with open(out) as f:
            return f.read()


def _functions(asm, pattern):
    """(mangled name, instruction lines) of every function whose name matches pattern."""
    for m in re.finditer(r"^(_Z\S*(?:%s)\S*):" % pattern, asm, re.M):
        end = asm.index(".Lfunc_end", m.end())
        yield m.group(1), [ln.strip() for ln in asm[m.end():end].split("\n")]


@pytest.mark.slow
@pytest.mark.parametrize("src", ["lbm_kernels.hip", "lbm3d_kernels.hip"])
def test_step_kernel_stores_are_nontemporal(src):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    asm = _device_asm(src)
    checked = 0
    excepted = 0
    bad = []
    for m in re.finditer(r"^(_Z\S*k_step\S*):", asm, re.M):
        name = m.group(1)
        end = asm.index(".Lfunc_end", m.end())
        plain = []
        for line in asm[m.end():end].split("\n"):
            ins = line.strip()
            if ins.startswith("global_store"):
                checked += 1
                if not re.search(r"\bnt\b", ins):
                    plain.append((name, ins))
        if "k_step3_aa_odd" in name and "Shifted" in name:
            excepted += 1
            if len(plain) != 10:
                bad.append((name, f"{len(plain)} plain stores, expected the 10 with c_x != 0"))
        else:
            bad.extend(plain)
    assert checked > 0
    if src == "lbm3d_kernels.hip":
        assert excepted > 0
    assert not bad, bad[:5]


@pytest.mark.slow
@pytest.mark.parametrize("src,pattern,storage,want", [
    ("lbm_kernels.hip", "k_step_dense_aaI", "3F64", 9),
    ("lbm3d_kernels.hip", "k_step3_aaI", "", 19),
])
def test_aa_even_loads_are_nontemporal(src, pattern, storage, want):
    """Even AA instantiations (last template flag false: mangled ...Lb0EEEv) issue exactly
    `want` nontemporal global loads, their own slots."""
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    seen = 0
    bad = []
    for name, lines in _functions(_device_asm(src), pattern):
        if storage not in name or "Lb0EEEv" not in name:
            continue
        seen += 1
        nt = sum(1 for ins in lines if ins.startswith("global_load") and re.search(r"\bnt\b", ins))
        if nt != want:
            bad.append((name, nt))
    assert seen > 0
    assert not bad, bad[:5]
