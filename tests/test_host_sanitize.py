"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU, no GPU): every source of libfdwave.so compiled for the host only, linked
with a host-memory stand-in for the HIP runtime (tests/hostcheck/fake_hip.hip)
and a driver that calls every entry point (tests/hostcheck/driver.cpp):
forward sweeps of every variant, points on and between nodes (staged, routed
and heavy tables), adjoint, checkpointed and whole-axis gradients, Born
modelling, the autotuner, forward and gradient batches with and without graph
capture, and error paths (among them a two-level exchange pass whose wait ran
out, which the stand-in forces by setting the pass's error word: the call must
return FD_ESYNC, and the next call on the same workspace must clear it).

Besides the sanitizers' own checks, the stand-in checks every sweep kernel's
arguments (single-pass and every entry of a grouped launch's table) against
the buffers the caller passed, the tile counts against the grid, the rows each
time level injects or records, the capacity of staged point walks, exchange
passes' residency, counter capacity and epochs, every fill kernel's range
(fills run for real), stream and event lifetimes, and graph capture's
fork/join rules; a batch must release every event and graph it creates."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def hostcheck_exe(tmp_path_factory):
    import importlib.util

    spec = importlib.util.spec_from_file_location("hostcheck_build", os.path.join(HERE, "hostcheck", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.build(str(tmp_path_factory.mktemp("hostcheck")), jobs=min(8, os.cpu_count() or 1))


def test_host_code_is_clean_under_sanitizers(hostcheck_exe, tmp_path):
    env = dict(os.environ)
    env["FD_AUTOTUNE_CACHE"] = str(tmp_path / "tune.txt")  # the driver's tuner call writes here
    # the library keeps its lane streams for the life of the process by design
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([hostcheck_exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-3000:])
    print(r.stderr[-6000:])
    assert r.returncode == 0, r.stderr[-6000:]
    assert "hostcheck errors 0 warnings 0, unexpected status 0" in r.stdout
    assert "live events and graphs 0" in r.stdout
    assert "Sanitizer" not in r.stderr
    ok = sum(1 for line in r.stdout.splitlines() if line.startswith("ok "))
    assert ok >= 40, ok
