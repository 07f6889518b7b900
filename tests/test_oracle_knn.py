"""Pins of the oracle stencil selection (Sec. 2.1): brute force, hand-derived ties."""
import numpy as np
import pytest

import nodesets as ns
from oracle import knn


def lattice5():
    """5x5 lattice with coordinates (integer * 2^-10): every key is exact."""
    g = np.array([(i, j) for i in range(5) for j in range(5)], dtype=np.float64) * 2.0 ** -10
    return g  # node id = 5*i + j, centre = 12


def test_lattice_ties_hand_derived():
    """Hand-derived stencils of tests/golden/lattice_ties.txt (5x5 lattice, exact keys)."""
    import os
    X = lattice5()
    cases = 0
    with open(os.path.join(os.path.dirname(__file__), "golden", "lattice_ties.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            head, st = line.split(":")
            c, n = (int(t) for t in head.split())
            off, idx = knn.knn_bruteforce(X, n)
            assert idx[off[c]:off[c + 1]].tolist() == [int(t) for t in st.split()], line
            off2, idx2 = knn.knn_exact(X, n)
            assert np.array_equal(idx, idx2)
            cases += 1
    assert cases == 3


def test_self_first_with_duplicate_node():
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 0.0], [0.0, 2.0]])
    off, idx = knn.knn_bruteforce(X, 3)
    assert idx[0:3].tolist() == [0, 2, 1]      # node 2 duplicates node 0: key 0, after self
    assert idx[6:9].tolist() == [2, 0, 1]
    off2, idx2 = knn.knn_exact(X, 3)
    assert np.array_equal(idx, idx2)


def test_key_is_left_to_right_sum_of_squares():
    X = np.array([[0.1, 0.2, 0.3], [0.7, -0.4, 1.9]])
    k = knn.sq_key(X, 0, np.array([1]))[0]
    dx, dy, dz = 0.7 - 0.1, -0.4 - 0.2, 1.9 - 0.3
    assert k == (dx * dx + dy * dy) + dz * dz


@pytest.mark.parametrize("case", ["disk", "cube", "varsize"])
def test_tree_equals_bruteforce(case):
    if case == "disk":
        X = ns.disk(0.0404, 1001).X
        sizes = 15
    elif case == "cube":
        X = ns.cube_minus_sphere(1.0 / 14, 1002).X
        sizes = 35
    else:
        nd = ns.l_shape(0.03, 5)
        X = nd.X
        sizes = np.random.default_rng(3).integers(1, 71, size=nd.N)
    o1, i1 = knn.knn_bruteforce(X, sizes)
    o2, i2 = knn.knn_exact(X, sizes, extra=1)
    assert np.array_equal(o1, o2)
    assert np.array_equal(i1, i2)


def test_stencils_are_sorted_by_key_then_index():
    X = ns.torus(0.03, 9).X
    off, idx = knn.knn_exact(X, 20)
    for i in range(0, X.shape[0], 97):
        st = idx[off[i]:off[i + 1]]
        assert st[0] == i and len(set(st.tolist())) == 20
        k = knn.sq_key(X, i, st[1:])
        assert np.all((k[1:] > k[:-1]) | ((k[1:] == k[:-1]) & (st[2:] > st[1:-1])))
        # nothing outside the stencil is closer than its last member
        rest = np.setdiff1d(np.arange(X.shape[0]), st)
        kr = knn.sq_key(X, i, rest)
        assert np.all((kr > k[-1]) | ((kr == k[-1]) & (rest > st[-1])))
