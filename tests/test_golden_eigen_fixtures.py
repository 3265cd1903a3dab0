"""The committed oracle eigenvalue fixtures (tests/golden/eig_*.txt, written by
tests/golden/make_eigen_fixtures.py) parse, are complete and record a passed
independent check: k values in the order of the wanted end of the spectrum,
every stored residual within the oracle's tol 1e-12, status 0, and for the
random graphs ARPACK agreement within 1e-10, for the stencil the spectrum
slicing count equal to k."""
import glob
import os
import re

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FILES = sorted(glob.glob(os.path.join(GOLDEN, "eig_*.txt")))


def parse(path):
    head = [l[1:].strip() for l in open(path) if l.startswith("#")]
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    idx = np.array([int(r[0]) for r in rows])
    ev = np.array([float(r[1]) for r in rows])
    res = np.array([float(r[2]) for r in rows])
    return head, idx, ev, res


@pytest.mark.parametrize("path", FILES, ids=[os.path.basename(f) for f in FILES])
def test_fixture_is_complete_and_checked(path):
    head, idx, ev, res = parse(path)
    text = "\n".join(head)
    k = int(re.search(r"k = (\d+) (smallest|largest)", text).group(1))
    smallest = "smallest" in text
    assert np.array_equal(idx, np.arange(k)) and ev.size == k
    assert np.all(np.isfinite(ev))
    assert np.all(np.diff(ev) >= 0) if smallest else np.all(np.diff(ev) <= 0)
    assert "oracle status 0" in text
    assert np.all(res <= 1e-12)
    m = re.search(r"agrees to max \|dlambda\| / max\(1, \|lambda\|\) = ([0-9.eE+-]+)", text)
    s = re.search(r"(\d+) eigenvalues below sigma = \S+ \(expected (\d+)\)", text)
    assert m or s, "no independent check recorded"
    if m:
        assert float(m.group(1)) <= 1e-10
    if s:
        assert int(s.group(1)) == int(s.group(2)) == k
