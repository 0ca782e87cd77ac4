"""Builds libfizi.so (HIP, gfx950) in-tree with hipcc.

Each .hip source under csrc/ is compiled to an object in parallel and the
objects are linked into paper_1907_04393_amd/lib/libfizi.so. Packed FP32
instructions are disabled for device code (-packed-fp32-ops).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import hashlib
import json
import os
import struct
import subprocess
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libfizi.so")
HASHES = os.path.join(LIBDIR, "kernel_hashes.json")
READELF = "/opt/rocm/llvm/bin/llvm-readelf"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC,
         "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _compile(src, objdir):
    obj = os.path.join(objdir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def _code_objects(blob: bytes):
    """The gfx950 code objects of the offload bundles embedded in a built
    library (each bundle: a magic string, an entry count, then per entry its
    offset, size and target triple)."""
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    pos = 0
    while True:
        i = blob.find(magic, pos)
        if i < 0:
            return
        (n,) = struct.unpack_from("<Q", blob, i + len(magic))
        off = i + len(magic) + 8
        for _ in range(n):
            o, size, tlen = struct.unpack_from("<QQQ", blob, off)
            off += 24
            triple = blob[off:off + tlen].decode(errors="replace")
            off += tlen
            if size and triple.endswith(ARCH):
                yield blob[i + o:i + o + size]
        pos = i + 1


def kernel_hashes(lib_path: str = LIB) -> dict:
    """sha256 (first 16 hex digits) of every kernel's machine code and
    descriptor in the built library, keyed by symbol: measurements taken on
    one build (HBM byte counters) are tied to the code they were taken on.
    The descriptor's code entry offset (bytes 16-23, the distance to where
    the linker placed the code) is left out, so that a change to another
    kernel of the library does not change the hash."""
    blob = open(lib_path, "rb").read()
    out = {}
    for co in _code_objects(blob):
        with tempfile.NamedTemporaryFile(suffix=".co") as f:
            f.write(co)
            f.flush()
            txt = subprocess.run([READELF, "-sSW", f.name], capture_output=True, text=True).stdout
        secs, syms = {}, []
        for line in txt.splitlines():
            parts = line.split()
            if line.lstrip().startswith("[") and "]" in line:
                fields = line.split("]", 1)[1].split()
                if len(fields) >= 5 and fields[0].startswith("."):
                    try:
                        secs[fields[0]] = (int(fields[2], 16), int(fields[3], 16))
                    except ValueError:
                        pass
            elif len(parts) == 8 and parts[3] in ("FUNC", "OBJECT") and parts[0].endswith(":"):
                syms.append((parts[7], int(parts[1], 16), int(parts[2])))
        text, rodata = secs.get(".text"), secs.get(".rodata")
        for name, addr, size in syms:
            sec = text if not name.endswith(".kd") else rodata
            if sec is None or size == 0:
                continue
            start = sec[1] + (addr - sec[0])
            key = name[:-3] if name.endswith(".kd") else name
            data = bytearray(co[start:start + size])
            if name.endswith(".kd") and len(data) >= 24:
                data[16:24] = bytes(8)
            h = out.setdefault(key, hashlib.sha256())
            h.update(bytes(data))
    return {k: v.hexdigest()[:16] for k, v in sorted(out.items())}


def build(verbose: bool = False) -> str:
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(lambda s: _compile(s, objdir), srcs))
    objs = [o for o, _ in results]
    if verbose:
        for _, err in results:
            if err.strip():
                print(err)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    with open(HASHES, "w") as f:
        json.dump(kernel_hashes(LIB), f, indent=1)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
