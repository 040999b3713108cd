"""Pins of oracle.linbin (first step of Sec. 4) and oracle.grid (Eq. (16)).

* hand-derived fixture (tests/golden/linbin_tiny.txt), incl. the clamp at the
  last node, out-of-grid skipping and round-half-even of the 2^-40 quanta;
* mass: every point adds exactly 2^40;
* first moment: linear binning preserves each point's coordinates;
* second moment: along each axis the binned variance exceeds the data's by
  exactly f(1-f) delta^2 per point (what linear weights imply);
* a point on a node puts all its mass there.
"""
import os

import numpy as np
import pytest

from oracle import grid, linbin


def _read_fixture(path):
    cases = {}
    cur = None
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "case":
            cur = {"points": [], "counts": []}
            cases[tok[1]] = cur
        elif tok[0] == "grid":
            d = int(tok[1])
            M = [int(t) for t in tok[2:2 + d]]
            lo = [float.fromhex(t) for t in tok[2 + d:2 + 2 * d]]
            de = [float.fromhex(t) for t in tok[2 + 2 * d:2 + 3 * d]]
            cur["grid"] = {"d": d, "M": np.array(M), "P": 2 * np.array(M), "lo": np.array(lo), "delta": np.array(de)}
        elif tok[0] == "point":
            cur["points"].append([float.fromhex(t) for t in tok[1:]])
        elif tok[0] == "skipped":
            cur["skipped"] = int(tok[1])
        elif tok[0] == "count":
            cur["counts"].append((tuple(int(t) for t in tok[1:-1]), int(tok[-1])))
    return cases


def test_golden_fixture(repo_root):
    cases = _read_fixture(os.path.join(repo_root, "tests", "golden", "linbin_tiny.txt"))
    assert set(cases) == {"A", "B"}
    for name, c in cases.items():
        counts, skipped = linbin.linbin(np.array(c["points"]), c["grid"])
        want = np.zeros(counts.shape, dtype=np.int64)
        for idx, v in c["counts"]:
            want[idx] += v
        np.testing.assert_array_equal(counts, want, err_msg=name)
        assert skipped == c["skipped"]


def _random_case(d, n, seed, M=None):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((d, d))
    X = rng.standard_normal((n, d)) @ A.T
    G = 0.2 * np.eye(d)
    if M is None:
        M = [7 + 3 * k for k in range(d)]
    return X, grid.plan_auto(X, G, M)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_mass_exact(d):
    X, g = _random_case(d, 3000, d)
    counts, skipped = linbin.linbin(X, g)
    assert skipped == 0
    assert int(counts.sum()) == X.shape[0] << 40
    assert counts.min() >= 0


@pytest.mark.parametrize("d", [1, 2, 3])
def test_first_and_second_moment(d):
    X, g = _random_case(d, 2000, 10 + d)
    counts, _ = linbin.linbin(X, g)
    c = linbin.counts_to_real(counts)
    n = X.shape[0]
    for k in range(d):
        nodes = grid.nodes(g, k)
        shape = [1] * d
        shape[k] = -1
        gk = nodes.reshape(shape)
        m1 = float((c * gk).sum())
        tol = n * (2 ** d) * 2.0 ** -40 * (abs(g["lo"][k]) + g["M"][k] * g["delta"][k]) + 1e-9
        assert abs(m1 - X[:, k].sum()) <= tol
        t = (X[:, k] - g["lo"][k]) / g["delta"][k]
        f = t - np.floor(t)
        excess = float((f * (1 - f)).sum()) * g["delta"][k] ** 2
        m2 = float((c * gk * gk).sum())
        assert m2 == pytest.approx(float((X[:, k] ** 2).sum()) + excess, rel=1e-9)


def test_point_on_node():
    g = grid.plan([-1.0, 2.0], [1.0, 6.0], [5, 9])       # delta = (0.5, 0.5)
    X = np.array([[-0.5, 3.5], [1.0, 6.0], [-1.0, 2.0]])
    counts, skipped = linbin.linbin(X, g)
    assert skipped == 0
    assert counts[1, 3] == 1 << 40
    assert counts[4, 8] == 1 << 40
    assert counts[0, 0] == 1 << 40
    assert int(counts.sum()) == 3 << 40


def test_out_of_grid_skipped():
    g = grid.plan([0.0], [1.0], [5])
    X = np.array([[-1e-9], [0.5], [1.0 + 1e-9], [1.0]])
    counts, skipped = linbin.linbin(X, g)
    assert skipped == 2
    assert int(counts.sum()) == 2 << 40


def test_grid_plan_bits():
    X = np.array([[0.1, -3.0], [2.5, 4.0]])
    G = np.array([[0.04, 0.01], [0.01, 0.09]])
    g = grid.plan_auto(X, G, [16, 32], pad_sd=4.0)
    assert g["lo"][0] == 0.1 - 4.0 * 0.2
    assert g["lo"][1] == -3.0 - 4.0 * 0.3
    assert g["delta"][0] == ((2.5 + 4.0 * 0.2) - (0.1 - 4.0 * 0.2)) / 15.0
    assert list(g["P"]) == [32, 64]
