"""CPU test of the GPU library's coarse stencil tables
(paper_2412_04980_amd/csrc/tables.hpp, Sec. 3.3 and Appendix A): a small driver
built with hipcc (host code only, no GPU) prints the tables of levels 2-6, which
must equal the oracle's independently computed stencils (oracle/stencils.py,
themselves pinned digit for digit to the printed ones) bit for bit, since both
round the same exact rational once.  The 1-D factors that the wide-stencil
kernels evaluate separably must rebuild the 2-D tables
(Laplace = t (x) m + m (x) t, wavenumber = m (x) m) and be symmetric, which the
kernels' tap loops assume."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import stencils

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def tables(tmp_path_factory):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("tables") / "tables_harness")
    subprocess.run([HIPCC, "-O2", "-std=c++17", os.path.join(ROOT, "tests", "tables_harness.cpp"),
                    "-o", exe], check=True, capture_output=True, timeout=300)
    vals = subprocess.run([exe], capture_output=True, text=True, check=True,
                          timeout=60).stdout.split()
    out, pos = {}, 0
    while pos < len(vals):
        level, R = int(vals[pos]), int(vals[pos + 1])
        pos += 2
        n = 2 * R + 1
        take = lambda k: np.array([float(v) for v in vals[pos:pos + k]])
        lap = take(n * n).reshape(n, n); pos += n * n
        wav = take(n * n).reshape(n, n); pos += n * n
        t1 = take(n); pos += n
        m1 = take(n); pos += n
        out[level] = (lap, wav, t1, m1)
    return out


@pytest.mark.parametrize("level", [2, 3, 4, 5, 6])
def test_tables_equal_the_oracle_stencils(tables, level):
    lap, wav, _, _ = tables[level]
    L, K = stencils.stencils_2d_float(level)
    assert lap.shape == L.shape and wav.shape == K.shape
    assert np.array_equal(lap, L)
    assert np.array_equal(wav, K)


@pytest.mark.parametrize("level", [2, 3, 4, 5, 6])
def test_separable_factors_rebuild_the_tables_and_are_symmetric(tables, level):
    lap, wav, t1, m1 = tables[level]
    assert np.array_equal(t1, t1[::-1]) and np.array_equal(m1, m1[::-1])
    scale = np.max(np.abs(lap))
    assert np.max(np.abs(np.outer(m1, t1) + np.outer(t1, m1) - lap)) <= 1e-15 * scale
    assert np.max(np.abs(np.outer(m1, m1) - wav)) <= 1e-15 * np.max(np.abs(wav))
