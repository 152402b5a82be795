"""The C ABI from C: a C99 program includes only include/fdwave.h, links
libfdwave.so and calls the host-only entry points (no GPU needed): version,
status strings, workspace sizing, the gradient storage choice and host-side
rejection of bad descriptors."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1707_02347_amd")

PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "fdwave.h"

int main(void)
{
    fd_grid g;
    memset(&g, 0, sizeof g);
    g.ndim = 3;
    g.space_order = 8;
    g.n[0] = 32; g.n[1] = 30; g.n[2] = 40;
    g.h[0] = g.h[1] = g.h[2] = 10.0;
    fd_time t = {100, 1e-3};
    int32_t idx[6] = {3, 4, 5, 10, 11, 12};
    fd_points rec;
    memset(&rec, 0, sizeof rec);
    rec.n = 2;
    rec.idx = idx;
    fd_options o;
    memset(&o, 0, sizeof o);
    size_t fwd = fd_workspace_size(&g, &t, NULL, &rec, NULL, FD_OP_FORWARD);
    size_t need = 0;
    int rc = fd_gradient_storage(&g, &t, NULL, &rec, FD_OP_GRADIENT, (size_t)1 << 40, &o, &need);
    fd_options full;
    memset(&full, 0, sizeof full);
    full.ckpt_every = 100;
    size_t fsz = fd_workspace_size(&g, &t, NULL, &rec, &full, FD_OP_GRADIENT);
    printf("version %d\n", fd_version());
    printf("fwd %zu\n", fwd);
    printf("storage %d %d %d\n", rc, o.ckpt_every, need == fsz);
    g.space_order = 7;
    printf("bad %d\n", fd_forward(&g, &t, (const float *)0x1000, NULL, NULL, NULL, NULL, NULL, 0, NULL, NULL));
    printf("str %s\n", fd_strerror(FD_EWORKSPACE));
    return 0;
}
"""


def test_c_program_links_and_calls_host_entry_points(tmp_path):
    if not os.path.exists(os.path.join(LIBDIR, "libfdwave.so")):
        pytest.skip("libfdwave.so is not built")
    src = tmp_path / "abi.c"
    src.write_text(PROGRAM)
    exe = tmp_path / "abi"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                           "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe),
                           "-L", LIBDIR, "-lfdwave", "-Wl,-rpath," + LIBDIR])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, check=True).stdout
    lines = dict(line.split(" ", 1) for line in out.strip().splitlines())
    assert lines["version"] == "100"
    assert int(lines["fwd"]) > 5 * 32 * 30 * 40 * 4
    assert lines["storage"] == "0 100 1"          # a budget that holds the whole axis stores it
    assert lines["bad"] == "-1"                    # FD_EINVAL before any device work
    assert len(lines["str"]) > 3
