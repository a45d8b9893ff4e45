"""The benchmark's command-line contract, checked without a GPU: a request
for more than one GPU ends with a message and a non-zero status before any
device work, the workloads parse, and the network workloads record the
source hash of the kernels they time."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_help_lists_every_workload():
    r = _bench("--help")
    assert r.returncode == 0
    for w in ("turbulence3d", "shockvortex2d", "ensemble2d", "learned64", "nnforward64", "nntrain64"):
        assert w in r.stdout


def test_source_hashes_are_stable_and_distinct():
    sys.path.insert(0, ROOT)
    import bench

    a, b = bench.kernel_source_hash(), bench.nn_source_hash()
    assert len(a) == 16 and len(b) == 16 and a != b
    assert a == bench.kernel_source_hash()
