"""Wait states ahead of the hand-written LDS DMA instructions (CPU only: reads
the gfx950 assembly that hipcc writes for this library's own kernels).

On gfx9 a vector-memory instruction that reads an SGPR written by a VALU
instruction needs 5 wait states in between, and an LDS DMA that reads M0 right
after a scalar write of M0 needs 1.  The compiler pads its own buffer loads for
both but treats inline assembly as opaque.  The stream kernel builds its buffer
resource with v_readfirstlane and issues the DMA as inline assembly, so every
DMA must carry its own padding; a DMA that reads a stale resource streams from
the wrong address (wrong values, or a memory fault).

For every `buffer_load ... lds` in the assembly, and for each SGPR it reads
(resource words, M0), the nearest earlier writer in the same basic block must
be a VALU at least 5 wait states back, or an SALU at least 1 wait state back
for M0.  A label (block join) reached within 5 wait states fails the check.
"""
import concurrent.futures as cf
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_07759_amd", "csrc")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")


def _sgprs(tok):
    m = re.match(r"s\[(\d+):(\d+)\]$", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"s(\d+)$", tok)
    if m:
        return {int(m.group(1))}
    return {"m0"} if tok == "m0" else set()


def _dest(ins):
    op = ins.split()[0]
    first = ins[len(op):].split(",")[0].strip()
    return _sgprs(first)


def _nearest_writer(lines, i, reg, limit=6):
    """(kind, wait states) of the nearest instruction before line i writing reg."""
    ws = 0
    j = i - 1
    while j >= 0 and ws < limit:
        t = lines[j].strip()
        j -= 1
        if not t or t.startswith(";") or t.startswith("."):
            continue
        if re.match(r"^[\w.$]+:", t):
            return "label", ws
        op = t.split()[0]
        if reg in _dest(t):
            return ("valu" if op.startswith("v_") else "salu"), ws
        ws += int(t.split()[1].rstrip(",")) + 1 if op == "s_nop" else 1
    return "far", ws


def hazards(asm_text):
    """Offending (line, register, writer kind, wait states) of an assembly file."""
    lines = asm_text.split("\n")
    bad = []
    n_dma = 0
    for i, l in enumerate(lines):
        s = l.strip()
        if not (s.startswith("buffer_load") and "lds" in s.split()):
            continue
        n_dma += 1
        regs = {"m0"}
        for t in s.split(None, 1)[1].split(","):
            regs |= _sgprs(t.strip())
        for r in regs:
            kind, ws = _nearest_writer(lines, i, r)
            if (kind == "valu" and ws < 5) or (kind == "salu" and r == "m0" and ws < 1) or \
                    (kind == "label" and ws < 5):
                bad.append((i + 1, r, kind, ws))
    return n_dma, bad


def test_checker_flags_an_unpadded_dma():
    # the checker itself: a readfirstlane straight into the resource is a hazard,
    # the same sequence behind s_nop 4 is not
    unpadded = "\n".join(["v_readfirstlane_b32 s4, v2", "s_mov_b32 s7, s3", "s_nop 0",
                          "buffer_load_dword v1, s[4:7], 0 offen lds"])
    padded = unpadded.replace("s_nop 0", "s_nop 4")
    assert hazards(unpadded)[1] and not hazards(padded)[1]
    m0 = "\n".join(["s_mov_b32 m0, s9", "buffer_load_dword v1, s[4:7], 0 offen lds"])
    assert hazards(m0)[1]


def _asm(src, out_dir):
    out = os.path.join(out_dir, os.path.basename(src) + ".s")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++20", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-x", "hip",
           "-S", "--cuda-device-only", src, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_every_lds_dma_is_padded(tmp_path):
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        outs = list(ex.map(lambda s: _asm(s, str(tmp_path)), srcs))
    total = 0
    for o in outs:
        n, bad = hazards(open(o).read())
        total += n
        assert not bad, f"{os.path.basename(o)}: {bad[:5]}"
    assert total > 0   # the stream kernels do hold LDS DMA
