"""The device code the library ships (gfx950 code objects embedded in
libfgraft.so, disassembled with the ROCm LLVM tools): no float64
instruction anywhere (the precision form keeps every device computation in
float32 or narrower; float64 exists only in the oracle on the host), no
packed-float32 VALU instruction (the build disables them), and every kernel
keeping float32 subnormals (its descriptor's float32 denormal mode is 3, no
flushing: the screen margins bound an underflowing operation's error by
2^-150, which flushing to zero would exceed).  The extraction and the
disassembly run in a child process that reports a small summary."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2609_30493_amd", "libfgraft.so")
OBJDUMP = "/opt/rocm/llvm/bin/llvm-objdump"

# Reads every offload bundle in the .hip_fatbin section, keeps the gfx950
# entries, disassembles them and reports the mnemonics the checks need.
_CHILD = r'''
import json, os, re, struct, subprocess, sys, tempfile
lib, objdump = sys.argv[1], sys.argv[2]
tmp = tempfile.mkdtemp()
fat = os.path.join(tmp, "fatbin.bin")
subprocess.run(["objcopy", "--dump-section", ".hip_fatbin=" + fat, lib], check=True, capture_output=True)
data = open(fat, "rb").read()
magic = b"__CLANG_OFFLOAD_BUNDLE__"
cos, pos = [], 0
while True:
    i = data.find(magic, pos)
    if i < 0:
        break
    count = struct.unpack_from("<Q", data, i + len(magic))[0]
    p = i + len(magic) + 8
    for _ in range(count):
        off, size, tlen = struct.unpack_from("<QQQ", data, p)
        p += 24
        triple = data[p:p + tlen].decode()
        p += tlen
        if triple.endswith("gfx950"):
            path = os.path.join(tmp, "co%d.o" % len(cos))
            open(path, "wb").write(data[i + off:i + off + size])
            cos.append(path)
    pos = i + 1
RE = os.path.join(os.path.dirname(objdump), "llvm-readelf")
kernels, f64, pk = set(), set(), set()
denorm32 = {}
for co in cos:
    # kernel descriptors (64 bytes, in .rodata): compute_pgm_rsrc1 at byte 48,
    # float32 denormal mode in its bits 16-17
    blob = open(co, "rb").read()
    secs = {}  # section index -> (address, file offset)
    for l in subprocess.run([RE, "-S", "-W", co], check=True, capture_output=True, text=True).stdout.splitlines():
        m = re.match(r"\s*\[\s*(\d+)\]\s+(\S+)\s+\S+\s+([0-9a-f]+)\s+([0-9a-f]+)", l)
        if m:
            secs[m.group(1)] = (int(m.group(3), 16), int(m.group(4), 16))
    for l in subprocess.run([RE, "--symbols", "-W", co], check=True, capture_output=True, text=True).stdout.splitlines():
        f = l.split()
        if len(f) >= 8 and f[-1].endswith(".kd"):
            addr, off = secs[f[6]]
            rs1 = struct.unpack_from("<I", blob, off + int(f[1], 16) - addr + 48)[0]
            m = str((rs1 >> 16) & 3)
            denorm32[m] = denorm32.get(m, 0) + 1
    out = subprocess.run([objdump, "-d", "--mcpu=gfx950", co], check=True, capture_output=True, text=True).stdout
    for name in ("k_beam", "k_make_screen", "k_leaf_knn", "k_finalize", "k_sat_"):
        if name in out:
            kernels.add(name)
    f64.update(re.findall(r"\b[sv]_[a-z0-9_]*f64[a-z0-9_]*", out))
    pk.update(re.findall(r"\bv_pk_(?:add|mul|fma)_f32\b", out))
print(json.dumps({"code_objects": len(cos), "kernels": sorted(kernels), "f64": sorted(f64), "pk": sorted(pk),
                  "denorm32": denorm32}))
'''


@pytest.fixture(scope="module")
def summary():
    if not (os.path.exists(OBJDUMP) and shutil.which("objcopy")):
        pytest.skip("ROCm llvm-objdump or binutils objcopy missing")
    assert os.path.exists(LIB), "build the library first"
    r = subprocess.run([sys.executable, "-c", _CHILD, LIB, OBJDUMP], check=True, capture_output=True, text=True)
    return json.loads(r.stdout)


def test_kernels_are_present(summary):
    assert summary["code_objects"] > 0
    assert summary["kernels"] == sorted(["k_beam", "k_make_screen", "k_leaf_knn", "k_finalize", "k_sat_"])


def test_no_float64_on_the_device(summary):
    assert not summary["f64"], summary["f64"]


def test_no_packed_float32_instructions(summary):
    assert not summary["pk"], summary["pk"]


def test_float32_subnormals_are_kept(summary):
    modes = summary["denorm32"]
    assert sum(modes.values()) >= 100, modes  # every kernel's descriptor was read
    assert set(modes) == {"3"}, modes
