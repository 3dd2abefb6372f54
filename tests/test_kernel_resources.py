"""Resource check of the device code (CPU only: hipcc cross-compiles gfx950).

A data kernel that combined a returning global atomic with heavy register
spills to scratch gave wrong, run-to-run different results on the MI355X,
while the same source with fewer spills, or with spills and no atomic, was
correct and bitwise reproducible.  No kernel of the library may combine the
two: every kernel that issues a global atomic must run without scratch."""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_cs_0101018_amd", "csrc")


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.fixture(scope="module")
def device_asm():
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found")
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "k.s")
        cmd = [hipcc, "-x", "hip", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-O3", "-std=c++17", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"),
               "-I", CSRC, "-ffp-contract=off", "--cuda-device-only", "-S",
               os.path.join(CSRC, "gpcg_kernels.hip"), "-o", out]
        r = subprocess.run(cmd, stderr=subprocess.PIPE, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return open(out).read()


def _kernels(asm):
    meta = {m.group(1): m.group(2)
            for m in re.finditer(r"\.amdhsa_kernel (\S+)\n(.*?)\.end_amdhsa_kernel", asm, re.S)}
    starts = [(m.start(), m.group(1)) for m in re.finditer(r"^(_Z\S+):", asm, re.M)]
    for i, (pos, name) in enumerate(starts):
        if name not in meta:
            continue
        end = starts[i + 1][0] if i + 1 < len(starts) else len(asm)
        scratch = int(re.search(r"amdhsa_private_segment_fixed_size (\d+)", meta[name]).group(1))
        yield name, scratch, len(re.findall(r"\b(?:global|flat|buffer)_atomic_", asm[pos:end]))


def test_no_kernel_combines_atomics_with_scratch(device_asm):
    ks = list(_kernels(device_asm))
    assert len(ks) > 50  # every kernel variant was found
    assert any(a for _, _, a in ks)  # the transition and persistent kernels use atomics
    bad = [(n, s, a) for n, s, a in ks if a and s]
    assert not bad, bad
