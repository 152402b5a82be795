"""Build libfdwave.so for gfx950 in-tree with hipcc.

Every .hip source in this directory, plus one generated source per kernel
configuration listed in fd_stream_configs.h (and the generated registry of
those configurations), is compiled to an object in parallel, then linked into
``paper_1707_02347_amd/libfdwave.so``.  Flags:

* ``--offload-arch=gfx950``: MI355X only.
* ``-ffp-contract=off``: no implicit FMA contraction; the kernels write every
  fused multiply-add explicitly so that all variants share one rounding order.
* ``-Xclang -target-feature -Xclang -packed-fp32-ops``: no packed FP32 VALU
  instructions.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
OUT = os.path.join(PKG, "libfdwave.so")
BUILD = os.path.join(PKG, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


GEN = os.path.join(BUILD, "gen")


def configs():
    """(M, T, PY, NW, MODE, F) tuples of every X(...) entry in fd_stream_configs.h."""
    text = open(os.path.join(HERE, "fd_stream_configs.h")).read()
    text = text.replace("FDW_AG", "3").replace("FDW_A", "1").replace("FDW_G", "2")
    out = []
    for m in re.finditer(r"X\((\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+)\)", text):
        out.append(tuple(int(g) for g in m.groups()))
    if len(set(out)) != len(out):
        raise RuntimeError("duplicate kernel configuration in fd_stream_configs.h")
    return out


def wave_configs():
    """(M, PY, NW) tuples of every W(...) entry in fd_stream_configs.h."""
    text = open(os.path.join(HERE, "fd_stream_configs.h")).read()
    out = [tuple(int(g) for g in m.groups()) for m in re.finditer(r"W\((\d+),\s*(\d+),\s*(\d+)\)", text)]
    if len(set(out)) != len(out):
        raise RuntimeError("duplicate wave configuration in fd_stream_configs.h")
    return out


def _write_if_changed(path, text):
    if os.path.exists(path) and open(path).read() == text:
        return
    with open(path, "w") as f:
        f.write(text)


def generate():
    """One source per configuration and the registry; returns their paths."""
    os.makedirs(GEN, exist_ok=True)
    paths, names = [], []
    for cfg in configs():
        name = "kEntry_%d_%d_%d_%d_%d" % cfg[:5]
        names.append(name)
        args = "%d, %d, %d, %d, %d, %d" % cfg
        text = ('// generated from fd_stream_configs.h\n#include "%s/fd_stream.h"\n#include "%s/fd_stream_entry.h"\n'
                "namespace fdw {\nextern StreamEntry %s;\nStreamEntry %s = {%s, &entry_launch<%s>,\n"
                "    &entry_launch_group<%s>, &entry_occupancy<%s>};\n}  // namespace fdw\n"
                % (HERE, HERE, name, name, args, args, args, args))
        path = os.path.join(GEN, name + ".hip")
        _write_if_changed(path, text)
        paths.append(path)
    wnames = []
    for cfg in wave_configs():
        name = "kWave_%d_%d_%d" % cfg
        wnames.append(name)
        args = "%d, %d, %d" % cfg
        text = ('// generated from fd_stream_configs.h\n#include "%s/fd_wave.h"\n#include "%s/fd_stream_entry.h"\n'
                "namespace fdw {\nextern WaveEntry %s;\nWaveEntry %s = {%s, &wave_launch<%s>, &wave_occupancy<%s>};\n"
                "}  // namespace fdw\n" % (HERE, HERE, name, name, args, args, args))
        path = os.path.join(GEN, name + ".hip")
        _write_if_changed(path, text)
        paths.append(path)
    reg = ['// generated from fd_stream_configs.h', '#include "%s/fd_stream_entry.h"' % HERE, "namespace fdw {"]
    reg += ["extern StreamEntry %s;" % n for n in names]
    reg += ["extern WaveEntry %s;" % n for n in wnames]
    reg += ["static const StreamEntry *const kRegistry[] = {"] + ["    &%s," % n for n in names] + ["};"]
    reg += ["static const WaveEntry *const kWaveRegistry[] = {"] + ["    &%s," % n for n in wnames] + ["};"]
    reg += ["const StreamEntry *const *stream_registry(int *count)", "{",
            "    *count = (int)(sizeof(kRegistry) / sizeof(kRegistry[0]));", "    return kRegistry;", "}",
            "const WaveEntry *const *wave_registry(int *count)", "{",
            "    *count = (int)(sizeof(kWaveRegistry) / sizeof(kWaveRegistry[0]));", "    return kWaveRegistry;", "}",
            "}  // namespace fdw", ""]
    path = os.path.join(GEN, "fd_registry.hip")
    _write_if_changed(path, "\n".join(reg))
    paths.append(path)
    for f in os.listdir(GEN):  # sources of configurations no longer listed
        if f.startswith(("kEntry_", "kWave_")) and os.path.join(GEN, f) not in paths:
            os.remove(os.path.join(GEN, f))
    return paths


def sources():
    own = sorted(os.path.join(HERE, f) for f in os.listdir(HERE) if f.endswith(".hip"))
    return own + generate()


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    deps = [src] + [os.path.join(HERE, f) for f in os.listdir(HERE) if f.endswith(".h")]
    if os.path.exists(obj) and os.path.getmtime(obj) > max(os.path.getmtime(d) for d in deps):
        return obj
    kernel = os.path.basename(src).startswith(("kEntry", "kWave"))
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    if kernel:
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if kernel:
        # a sweep kernel that spills registers to scratch memory is far slower
        # than any compiled alternative: refuse to ship it
        spills = [int(m) for m in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", r.stderr)]
        if any(spills):
            os.remove(obj)
            raise RuntimeError(f"{os.path.basename(src)}: kernel uses {max(spills)} bytes of scratch "
                               "per lane (register spills); drop or change this configuration")
    return obj


def build(jobs: int | None = None, verbose: bool = False, clean: bool = False) -> str:
    """Compile and link; objects newer than their sources and headers are reused
    unless clean=True."""
    os.makedirs(BUILD, exist_ok=True)
    if clean:
        for f in os.listdir(BUILD):
            if f.endswith(".o"):
                os.remove(os.path.join(BUILD, f))
    srcs = sources()
    # longest compiles first: generated kernel files
    srcs.sort(key=lambda p: (0 if os.path.basename(p).startswith(("kEntry", "kWave")) else 1, p))
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
