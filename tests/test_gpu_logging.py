"""TPCF_LOG_LEVEL on the GPU path: at level 3 a child process that stages a catalogue, autotunes
and computes zeta reports the catalogue, every device allocation, every autotuner configuration
and one line per compute call whose pair count is the one tpcf_get_stats returns."""
import os
import re
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = """
import catalogs
import paper_2604_08855_amd as tpcf
cat = catalogs.uniform(5000, 100.0, 3)
c = tpcf.Context(0)
c.set_bins(8, 2.0, 20.0, 4)
c.set_precision("mixed")
c.set_catalog(cat.x, cat.y, cat.z, None, box=cat.box, periodic=True)
c.autotune(0.5)
c.compute_zeta()
print("PAIRS", c.stats()["n_pairs"], flush=True)
"""


def test_log_level_3_reports_stages():
    env = dict(os.environ, TPCF_LOG_LEVEL="3")
    env.pop("TPCF_LOG_FILE", None)
    out = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr[-3000:]
    err = out.stderr
    assert "tpcf[info] catalogue: 5000 points in 1 catalogue(s), inputs in host memory" in err
    assert "tpcf[debug] device buffer: positions" in err
    assert len(re.findall(r"tpcf\[debug\] autotune: ", err)) == 20
    assert "tpcf[info] autotune: " in err
    pairs = int(re.search(r"PAIRS (\d+)", out.stdout).group(1))
    computes = re.findall(r"tpcf\[info\] compute: 1 catalogue\(s\), 5000 primaries, (\d+) pairs", err)
    assert computes and int(computes[-1]) == pairs
