"""CPU replay of the padding rule of the batched Newton-Schulz iteration.

Every submatrix is padded to a multiple of 32 with the identity, and the
padded block never mixes with the true one.  The prescaling X_0 = A_g / s_g
must not touch the padding: p(x) = x (3 - x^2) / 2 has the fixed point 1, but
a padded entry prescaled to 1/s_g leaves the basin [-sqrt(3), sqrt(3)] once
s_g < 1/sqrt(3) and grows without bound, and the infinite padded entry then
turns the true block into NaN through Inf * 0 in a dense product.  The replay
uses the two-product form of a step (W = 1.5 I - 0.5 X^2, X' = X W) in plain
numpy, FP64.
"""

import numpy as np

from waterbox import random_block_system


def _padded_sign(a, npad, prescale_padding, steps=60):
    n = a.shape[0]
    s = float(np.abs(a).sum(axis=1).max())
    x = np.eye(npad)
    x[:n, :n] = a / s
    if prescale_padding:
        x[n:, n:] /= s
    with np.errstate(over="ignore", invalid="ignore"):
        for _ in range(steps):
            w = 1.5 * np.eye(npad) - 0.5 * (x @ x)
            x = x @ w
    return s, x[:n, :n]


def test_padding_identity_is_a_fixed_point_under_small_scales():
    base = random_block_system(41, [13, 5, 5, 7, 3, 11], density=0.6, coupling=0.04, groups="all", mu=0.0)
    a = base.to_dense() * 0.2
    n = a.shape[0]
    npad = (n + 31) // 32 * 32
    assert npad > n
    lam, q = np.linalg.eigh(a)
    sign = (q * np.sign(lam)) @ q.T
    s, x_ok = _padded_sign(a, npad, prescale_padding=False)
    assert s < 1 / np.sqrt(5)
    assert np.abs(x_ok - sign).max() <= 1e-12
    _, x_bad = _padded_sign(a, npad, prescale_padding=True)
    assert not np.all(np.isfinite(x_bad))
