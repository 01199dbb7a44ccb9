"""Every kernel of libnmf compiles for gfx950 without scratch (private)
memory: register spills or dynamically indexed local arrays would put
per-lane scratch on the hot path.  Uses the compiler's resource-usage
remarks; runs on the CPU (hipcc cross-compiles)."""
import glob
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1509_09313_amd import build as B  # noqa: E402

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc is not installed")


def kernel_resources(src):
    cmd = ["hipcc", *B.flags_for(src), "--cuda-device-only", "-c", src, "-o", os.devnull,
           "-Rpass-analysis=kernel-resource-usage"]
    out = subprocess.run(cmd, capture_output=True, text=True)
    assert out.returncode == 0, out.stderr[-2000:]
    res, name = {}, None
    for line in out.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            res[name] = {}
        m = re.search(r"(ScratchSize \[bytes/lane\]|VGPRs): (\d+)", line)
        if m and name:
            res[name][m.group(1)] = int(m.group(2))
    return res


SOURCES = sorted(glob.glob(os.path.join(ROOT, "paper_1509_09313_amd", "csrc", "*.hip")))


@pytest.fixture(scope="module")
def resources():
    """Resource usage of every source, compiled in parallel once."""
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        return dict(zip(SOURCES, ex.map(kernel_resources, SOURCES)))


@pytest.mark.parametrize("src", SOURCES, ids=os.path.basename)
def test_no_scratch(src, resources):
    res = resources[src]
    if not res:   # a dispatch-only source (its kernels are instantiated elsewhere)
        with open(src) as fh:
            assert "__global__" not in fh.read(), f"no kernels reported for {src}"
        pytest.skip("no kernels in this file")
    spills = {k: v for k, v in res.items() if v.get("ScratchSize [bytes/lane]", 0) != 0}
    assert not spills, spills
