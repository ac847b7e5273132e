"""Resource guard for the gfx950 kernels (CPU: compiles, does not run them).

Builds every HIP source of the library with -save-temps and reads the AMD code-object
metadata of this build: no kernel may use scratch (private) memory -- a
spilled staging array silently costs ~25% of the forward kernel's time -- and
no packed-FP32 instruction may appear in the generated code.
"""
import os
import re
import subprocess

import pytest

from paper_2408_02758_amd import build as B


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    """The gfx950 assembly of every HIP source of the library, concatenated."""
    out = []
    for src in (s for s in B.SOURCES if s.endswith(".hip")):
        d = tmp_path_factory.mktemp("isa")
        cmd = [B.hipcc()] + B.HIPCC_FLAGS + ["-I", B.CSRC, "-save-temps", "-c", src, "-o", str(d / "k.o")]
        subprocess.run(cmd, check=True, cwd=d, stderr=subprocess.DEVNULL)
        s = [f for f in os.listdir(d) if f.endswith("gfx950.s")]
        assert s, f"no gfx950 assembly produced for {src}"
        out.append(open(d / s[0]).read())
    return out


def test_no_scratch(asm):
    kernels = 0
    for text in asm:
        meta = text[text.index("amdhsa.kernels:"):]
        for blk in meta.split("  - .")[1:]:
            name = re.search(r"\.name:\s+(\S+)", blk)
            if not name or "kernel" not in name.group(1):
                continue
            kernels += 1
            scratch = int(re.search(r"\.private_segment_fixed_size:\s+(\d+)", blk).group(1))
            assert scratch == 0, f"{name.group(1)} uses {scratch} bytes of scratch per lane"
    assert kernels >= 64


def test_no_packed_fp32(asm):
    for text in asm:
        assert not re.search(r"v_pk_(fma|mul|add)_f32", text)
