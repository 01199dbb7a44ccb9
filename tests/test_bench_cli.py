"""bench.py's command-line contract, on the CPU: the defaults, the modes,
and the refusal of more than one GPU (this library has no multi-GPU path)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_defaults():
    a = bench.parse([])
    assert (a.gpus, a.steps, a.warmup) == (1, 3, 1)
    assert (a.m, a.n, a.k, a.iters, a.cold_iters) == (1_000_000, 2_400, 30, 50, 5)
    assert not (a.sparse or a.dense or a.ksweep or a.pmc or a.pmc_bpp)


def test_modes_parse():
    for flag in ("--sparse", "--dense", "--ksweep", "--pmc", "--pmc-bpp"):
        a = bench.parse([flag])
        assert getattr(a, flag[2:].replace("-", "_"))


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, cwd=ROOT, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
    assert out.stdout == ""
