"""CPU pins of the third-order Pade sign map p(x) = x (15 - 10 x^2 + 3 x^4) / 8
(the iteration of the paper's GPU runs, Sec. VI-A), as the oracle evaluates it.

What fixes it, independently of its formula: p is odd with fixed points 0 and
+-1; its derivative is 15 (1 - x^2)^2 / 8 (so p'(0) = 15/8 and the fixed points
+-1 are of third order: 1 - p(1 - e) = (5/2) e^3 + O(e^4)); on (0, 1] the
composition converges to 1, i.e. to sign(x); and applied to a symmetric matrix
through matrix products (a textbook polynomial evaluation) the iteration
reaches the sign the Jacobi oracle computes from the eigendecomposition.
"""

import numpy as np

import oracle


def test_fixed_points_and_oddness():
    assert np.array_equal(oracle.pade_poly([0.0, 1.0, -1.0], 1), [0.0, 1.0, -1.0])
    x = np.linspace(-1.0, 1.0, 101)
    np.testing.assert_allclose(oracle.pade_poly(-x, 3), -oracle.pade_poly(x, 3), rtol=0, atol=1e-15)


def test_derivative_by_central_differences():
    x = np.linspace(-0.99, 0.99, 57)
    h = 1e-6
    fd = (oracle.pade_poly(x + h, 1) - oracle.pade_poly(x - h, 1)) / (2 * h)
    np.testing.assert_allclose(fd, 15.0 * (1.0 - x * x) ** 2 / 8.0, rtol=0, atol=1e-8)


def test_third_order_fixed_point():
    e = np.array([1e-2, 3e-3, 1e-3])
    err = 1.0 - oracle.pade_poly(1.0 - e, 1)
    np.testing.assert_allclose(err / e ** 3, 2.5, rtol=3e-2)


def test_composition_converges_to_sign():
    x = np.array([1e-3, 0.01, 0.3, 0.999, -0.05])
    y = oracle.pade_poly(x, 16)
    np.testing.assert_allclose(y, np.sign(x), rtol=0, atol=1e-14)
    # monotone on [0, 1]: more steps never move a value back toward 0
    z = np.linspace(0.0, 1.0, 201)
    assert np.all(np.diff(oracle.pade_poly(z, 2)) >= 0)


def test_matrix_iteration_reaches_the_jacobi_sign():
    rng = np.random.default_rng(5)
    n = 40
    g = rng.normal(size=(n, n))
    a = (g + g.T) / 2
    a += np.diag(np.where(np.arange(n) % 2 == 0, -3.0, 3.0))
    x = a / np.abs(a).sum(axis=1).max()
    for _ in range(30):
        x2 = x @ x
        x = x @ (15.0 * np.eye(n) - 10.0 * x2 + 3.0 * (x2 @ x2)) / 8.0
    np.testing.assert_allclose(x, oracle.dense_sign(a), rtol=0, atol=1e-12)
