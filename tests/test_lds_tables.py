"""The band builder's LDS staging tables (host code, no GPU): compiles a checker against the
builder with g++ and runs it.  For circles, spheres (centred and off-centre), a torus and
Dziuk's surface it checks, on every level and for every node, that each LDS address the
LDS-staged extension and fused sweep form lies in its workgroup's staged range and holds the
band index the gather form of the same pass reads (so the two forms read the same values), and
that the learned smoother's grouped patch rows address every present patch node (rows with
an absent middle node included) at the band index a search of the sorted grid keys finds, and
that the neighbour sum's segment tables give every listed node's band index and axis
neighbours, and that the tiled sweep's row tables stage, for every node, its stencil nodes and their Laplacian
neighbours at the band indices the extension and the neighbour sum read."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1307_4354_amd", "csrc")


def test_lds_staging_tables(tmp_path):
    exe = str(tmp_path / "lds_tables_check")
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-I" + CSRC,
           os.path.join(HERE, "lds_tables_check.cpp"), os.path.join(CSRC, "band_build.cpp"), "-o", exe]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        pytest.fail("build failed:\n" + r.stdout[-3000:])
    out = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=600)
    assert out.returncode == 0 and "ALL OK" in out.stdout, out.stdout[-3000:]
    # the neighbour sum's segment tables exist on every level
    assert all("sum segments 0 " not in ln for ln in out.stdout.splitlines() if "level" in ln)
    # the fused sweep's tables exist on the levels that have its addressing
    assert "sweep tables present" in out.stdout
    assert "patch groups 0," not in out.stdout.split("level 0:")[1].split("\n")[0]
    # rows whose middle node is absent (outer nodes present) occur and are addressed
    assert any("gapped rows 0," not in ln for ln in out.stdout.splitlines() if "gapped rows" in ln)
    # tiled-sweep tables exist on the large levels, and on every 3-D level when asked for
    assert any("tiles 0," not in ln for ln in out.stdout.splitlines() if "tiles" in ln)
    env = dict(os.environ, CPM_TILE_MIN_NODES="1000")
    out2 = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=600, env=env)
    assert out2.returncode == 0 and "ALL OK" in out2.stdout, out2.stdout[-3000:]
    # workgroups of 2 and 4 slots per thread (the large-level form), and the plain (z, y, x)
    # visit order instead of the Morton-blocked one
    for extra in ({"CPM_EXT_NPT": "4"}, {"CPM_EXT_NPT": "2", "CPM_MORTON_BITS": "-1"}):
        out3 = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=600,
                              env=dict(os.environ, **extra))
        assert out3.returncode == 0 and "ALL OK" in out3.stdout, (extra, out3.stdout[-3000:])
        assert "slots per thread %s" % extra["CPM_EXT_NPT"] in out3.stdout
