import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Automatic plans take the autotuner's cached choices, as in bench.py, so that
# the full-size tests run the configurations the benchmark times.
os.environ.setdefault("FD_AUTOTUNE_CACHE", os.path.join(ROOT, "paper_1707_02347_amd", "autotune_gfx950.txt"))

# GPU test files in the order they run: comparisons with the FP64 oracle
# first, so that a failure in a later file (which stops a run under -x)
# cannot hide them; batches, whose launches share the most host state,
# and the tuner, which changes the automatic plans of later calls, last.
# Files not listed keep their place among themselves after the listed ones.
ORDER = [
    "test_gpu_parity.py",
    "test_gpu_split.py",
    "test_gpu_wave.py",
    "test_gpu_random_configs.py",
    "test_gpu_offgrid.py",
    "test_gpu_sinc.py",
    "test_gpu_autograd.py",
    "test_gpu_born.py",
    "test_gpu_cache_policy.py",
    "test_gpu_batch.py",
    "test_gpu_autotune.py",
]


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")


def pytest_collection_modifyitems(session, config, items):
    def rank(item):
        name = os.path.basename(str(item.fspath))
        if name.startswith("test_zz"):
            return len(ORDER) + 1
        return ORDER.index(name) if name in ORDER else len(ORDER)

    items[:] = [it for _, it in sorted(enumerate(items), key=lambda p: (rank(p[1]), p[0]))]
