"""Host dense routines of the solver (dense.cpp), built with g++ into a small
harness: the eigenvectors that the recycle refresh takes for clustered
harmonic Ritz values.  Inverse iteration cannot separate eigenvalues closer
than its shift perturbation; the refresh needs the selected vectors to be
well conditioned (U = [..] P rho^{-1} inverts the triangular factor of G P),
so a cluster's vectors are kept mutually orthogonal."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1604_01713_amd", "csrc")


def test_clustered_eigenvalues_give_independent_vectors(tmp_path):
    exe = str(tmp_path / "cluster_eigvec")
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "host", "cluster_eigvec.cpp"), os.path.join(CSRC, "dense.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(r.stderr[-2000:])
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    print(out)
    m = re.search(r"R diag ratio ([0-9.e+-]+), max eigen-residual ([0-9.e+-]+)", out)
    ratio, res = float(m.group(1)), float(m.group(2))
    assert ratio > 1e-2      # the 16 vectors are far from dependent (2.7e-15 without the clusters)
    assert res < 1e-10       # and each is an eigenvector (|K| about 60)
