"""Pins of the reference Adam step (Kingma & Ba 2015, Alg. 1) used to check the
device's constant-optimisation step."""
import numpy as np

from oracle.constopt import adam_step


def _zeros(M, C):
    return np.zeros((M, C)), np.zeros((M, C))


def test_first_steps_move_by_lr_times_sign():
    # with a constant gradient the bias-corrected moments are g and g^2 exactly,
    # so every step moves each coordinate by lr * g / (|g| + eps)
    g = np.array([[3.0, -0.25, 1e-3, 0.0]])
    c = np.array([[1.0, 2.0, -1.0, 0.5]])
    m1, m2 = _zeros(1, 4)
    bc, bf = c.copy(), np.array([np.inf])
    lr = 0.01
    for t in range(1, 6):
        c1, m1, m2, bc, bf = adam_step(c, g, [1.0 / t], m1, m2, bc, bf, t, lr)
        np.testing.assert_allclose(c1 - c, -lr * g / (np.abs(g) + 1e-12), rtol=1e-12, atol=0)
        assert c1[0, 3] == c[0, 3]                    # zero gradient: no move
        c = c1


def test_best_point_and_revert():
    c = np.array([[1.0, 2.0], [3.0, 4.0], [5.0, 6.0]])
    g = np.ones((3, 2))
    m1, m2 = np.full((3, 2), 0.5), np.full((3, 2), 0.25)
    bc = np.array([[0.0, 0.0], [9.0, 9.0], [7.0, 7.0]])
    bf = np.array([2.0, 1.0, 1.0])
    c1, m1n, m2n, bc1, bf1 = adam_step(c, g, [1.5, 3.0, np.inf], m1, m2, bc, bf, 3, 0.1)
    # program 0 improved: its pre-step constants are recorded
    assert bf1[0] == 1.5 and np.array_equal(bc1[0], c[0]) and not np.array_equal(c1[0], c[0])
    # program 1 got worse: best unchanged, still steps
    assert bf1[1] == 1.0 and np.array_equal(bc1[1], bc[1]) and not np.array_equal(c1[1], c[1])
    # program 2 left the finite region: back to the best point, moments cleared
    assert np.array_equal(c1[2], bc[2]) and np.all(m1n[2] == 0) and np.all(m2n[2] == 0)


def test_minimises_a_quadratic():
    # f(c) = sum (c - c*)^2, gradient 2 (c - c*): Adam ends within about lr of c*
    target = np.array([[0.3, -1.7, 2.2]])
    c = np.zeros((1, 3))
    m1, m2 = _zeros(1, 3)
    bc, bf = c.copy(), np.array([np.inf])
    lr = 0.01
    for t in range(1, 2001):
        f = float(np.sum((c - target) ** 2))
        c, m1, m2, bc, bf = adam_step(c, 2 * (c - target), [f], m1, m2, bc, bf, t, lr)
    assert np.max(np.abs(c - target)) < 2 * lr
    assert bf[0] < 1e-4
