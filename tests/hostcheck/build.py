"""Build the host-code check: every source of libfdwave.so compiled for the host
only (no device code) with AddressSanitizer and UndefinedBehaviorSanitizer,
linked with the host-memory runtime stand-in (fake_hip.hip) and the driver
that calls every entry point (driver.cpp) into one executable.

Test infrastructure: the product library is built by
paper_1707_02347_amd/csrc/build.py; nothing here is part of it.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = "/opt/rocm/llvm/bin/clang++"
# sanitizers apply to host code only: each -fsanitize= follows -Xarch_host
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined"]
FLAGS = ["--offload-host-only", "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer",
         "-ffp-contract=off", "-Wno-unused-command-line-argument", *SAN]


def _sources():
    sys.path.insert(0, ROOT)
    from paper_1707_02347_amd.csrc import build as libbuild

    return libbuild.sources()


def _compile(args):
    src, obj = args
    if os.path.exists(obj) and os.path.getmtime(obj) > os.path.getmtime(src):
        heads = [os.path.join(ROOT, "paper_1707_02347_amd", "csrc", f)
                 for f in os.listdir(os.path.join(ROOT, "paper_1707_02347_amd", "csrc")) if f.endswith(".h")]
        if os.path.getmtime(obj) > max(os.path.getmtime(h) for h in heads):
            return obj
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed for {src}:\n{r.stderr[-4000:]}")
    return obj


def build(out_dir: str, jobs: int = 8) -> str:
    os.makedirs(out_dir, exist_ok=True)
    srcs = _sources() + [os.path.join(HERE, "fake_hip.hip")]
    pairs = [(s, os.path.join(out_dir, os.path.basename(s).rsplit(".", 1)[0] + ".o")) for s in srcs]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, pairs))
    drv = os.path.join(out_dir, "driver.o")
    r = subprocess.run([CLANGXX, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
                        "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                        "-c", os.path.join(HERE, "driver.cpp"), "-o", drv], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"driver compile failed:\n{r.stderr[-4000:]}")
    # the host-only objects still name their (absent) device images: define them
    stubs = set()
    for o in objs:
        nm = subprocess.run(["nm", "-u", o], capture_output=True, text=True).stdout
        stubs.update(line.split()[-1] for line in nm.splitlines() if "__hip_fatbin" in line)
    stub_c = os.path.join(out_dir, "fatbin_stubs.c")
    with open(stub_c, "w") as f:
        f.write("".join(f"char {s}[16];\n" for s in sorted(stubs)))
    exe = os.path.join(out_dir, "hostcheck")
    r = subprocess.run([CLANGXX, "-fsanitize=address,undefined", "-o", exe, drv, *objs, "-x", "c", stub_c],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    return exe


if __name__ == "__main__":
    exe = build(sys.argv[1] if len(sys.argv) > 1 else os.path.join(ROOT, "_work", "hostcheck"))
    sys.exit(subprocess.run([exe]).returncode)
