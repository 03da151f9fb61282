"""The benchmark's command line on a machine without a GPU: more than one GPU
is refused with a message, and every workload name is accepted by the
parser (the runs themselves need an MI355X)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_workload_names():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("spherical_voids_129", "diffuse_crack_257", "cantilever_193x97x97",
              "ellipsoidal_voids_amr_64x3", "j2_void_tension_128", "pf_mode1_4096",
              "pressurised_voids_129"):
        assert w in r.stdout
