"""Pins of the FP64 LRMSD oracle ("Loss function" section): the paper's
quaternion route (T matrix, largest eigenvalue, U from q) equals the Kabsch
SVD solution, the value is invariant under rigid motions of either structure
and zero for a rigid copy, and the input-side gradient matches central finite
differences and the translation/rotation invariances."""
import numpy as np
import pytest

from oracle import lrmsd as L


def _rot(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    return L.paper_U(q)


@pytest.mark.parametrize("n", [3, 7, 50, 400])
def test_quaternion_route_equals_kabsch(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, 3)) * 6 + 20
    y = rng.standard_normal((n, 3)) * 6 - 3
    a, K = L.kabsch(x, y)
    b, U, lam = L.quaternion(x, y)
    assert abs(a - b) < 1e-10 * max(1.0, a)
    # the paper's U maps the target onto the input: the transpose of Kabsch's
    assert np.max(np.abs(U - K.T)) < 1e-9
    assert abs(np.linalg.det(K) - 1.0) < 1e-12


def test_rigid_invariance_and_zero():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((60, 3)) * 8
    y = rng.standard_normal((60, 3)) * 8
    base = L.kabsch(x, y)[0]
    Q, t = _rot(rng), rng.standard_normal(3) * 30
    assert abs(L.kabsch(x, y @ Q.T + t)[0] - base) < 1e-10
    assert abs(L.kabsch(x @ Q.T - t, y)[0] - base) < 1e-10
    assert L.kabsch(x, x @ Q.T + t)[0] < 1e-9
    # a mirror image is not a rigid motion
    assert L.kabsch(x, x * np.array([1, 1, -1]))[0] > 1.0


def test_brute_force_rotation_search_is_not_better():
    """No sampled rotation does better than the solution (minimum is global)."""
    rng = np.random.default_rng(6)
    x = rng.standard_normal((25, 3)) * 4
    y = rng.standard_normal((25, 3)) * 4
    best, _ = L.kabsch(x, y)
    xc, yc = x - x.mean(0), y - y.mean(0)
    for _ in range(2000):
        Q = _rot(rng)
        val = np.sqrt(np.sum((xc - yc @ Q.T) ** 2) / len(x))
        assert val >= best - 1e-12


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    off = np.array([0, 9, 9, 30])
    x = rng.standard_normal((3, 30)) * 5
    y = rng.standard_normal((3, 30)) * 5
    go = np.array([0.7, 1.3, -2.0])
    g = L.lrmsd_grad_batch(x, y, off, go)
    h = 1e-6
    fd = np.zeros_like(y)
    for q in range(3):
        for a in range(30):
            y1 = y.copy(); y1[q, a] += h
            y2 = y.copy(); y2[q, a] -= h
            fd[q, a] = (np.dot(go, L.lrmsd_batch(x, y1, off)) -
                        np.dot(go, L.lrmsd_batch(x, y2, off))) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-7 * np.max(np.abs(g))
    # invariances of each chain's gradient
    for c in range(3):
        a0, a1 = off[c], off[c + 1]
        if a1 > a0:
            gc = g[:, a0:a1]
            assert np.max(np.abs(gc.sum(axis=1))) < 1e-10
            mom = np.cross(y[:, a0:a1].T, gc.T).sum(axis=0)
            assert np.max(np.abs(mom)) < 1e-9
