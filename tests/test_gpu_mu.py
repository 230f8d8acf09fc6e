"""GPU: frozen iteration, the mu tangent dN/dmu, and the mu search.

With the step counts k_g and scales s_g frozen, the electron count is the
polynomial map N_k(mu) = sum_g sum_l w_gl (1 - p_k((lam_gl - mu)/s_g))/2,
which the oracle evaluates from Jacobi eigenpairs.  Bars: N to 1e-9 (FP64
products, n <= 400), dN/dmu to 1e-7 relative, finite differences (central,
h = 1e-5) to 1e-6 relative, and the mu search to |N_k(mu*) - N_e| <= 1e-8
(the search tolerance) plus 1e-9 of rounding.
"""

import numpy as np
import pytest

from waterbox import water_config, block_offsets, water_system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smx():
    import paper_2004_10811_amd as smx
    smx.load_library()
    return smx


def frozen_ctx(smx, s, mu, steps=6):
    """Freeze an unconverged iteration (steps Newton-Schulz steps), where the
    map mu -> N is far from the step function and dN/dmu is O(1)."""
    ctx = smx.Context(0).load(s)
    ctx.configure(precision="fp64", mu=mu, max_iter=steps)
    ctx.evaluate(allow_not_converged=True)
    smx.smx_set_frozen(ctx.handle, True)
    return ctx


def n_and_slope(smx, ctx, mu):
    smx.smx_set_mu(ctx.handle, mu)
    r = ctx.evaluate()
    return r.n_elec, smx.smx_dn_dmu(ctx.handle)


def test_dn_dmu_matches_finite_differences(smx):
    s = water_config("water16")
    mu = 0.03
    ctx = frozen_ctx(smx, s, mu)
    n0, d0 = n_and_slope(smx, ctx, mu)
    h = 1e-5
    np_, _ = n_and_slope(smx, ctx, mu + h)
    nm, _ = n_and_slope(smx, ctx, mu - h)
    ctx.close()
    fd = (np_ - nm) / (2 * h)
    print(f"water16 frozen (6 steps): N = {n0:.10f}, dN/dmu = {d0:.6e}, FD = {fd:.6e}")
    assert d0 > 1.0
    assert abs(d0 - fd) <= 1e-6 * abs(d0) + 1e-9


def test_frozen_count_and_slope_match_oracle(smx, oracle_lib):
    s = water_system(n_mol=12, box=7.0, r_cut=3.5, seed=51)
    mu = -0.05
    ctx = frozen_ctx(smx, s, mu)
    info = ctx.group_info()
    n_gpu, d_gpu = n_and_slope(smx, ctx, mu + 0.01)
    ctx.close()
    spec = oracle_lib.GroupSpectra(s)
    n_or = spec.n_frozen(mu + 0.01, info["iters"], info["scale"])
    d_or = spec.dn_dmu_frozen(mu + 0.01, info["iters"], info["scale"])
    print(f"frozen N gpu {n_gpu:.12f} oracle {n_or:.12f}; dN/dmu gpu {d_gpu:.8e} oracle {d_or:.8e}")
    assert abs(n_gpu - n_or) <= 1e-9
    assert abs(d_gpu - d_or) <= 1e-7 * abs(d_or) + 1e-9
    assert np.all(info["iters"] == 6)


def test_find_mu_reaches_target(smx, oracle_lib):
    s = water_config("water16")
    ctx = smx.Context(0).load(s).configure(precision="fp64")
    target = s.n / 2
    mu, steps = smx.smx_find_mu(ctx.handle, target, 1e-8, 60)
    info = ctx.group_info()        # the last evaluation was the frozen one at mu
    ctx.close()
    spec = oracle_lib.GroupSpectra(s)
    n_or = spec.n_frozen(mu, info["iters"], info["scale"])
    print(f"water16 mu search: mu* = {mu:.10f} in {steps} evaluations; oracle N_k(mu*) - N_e = {n_or - target:.2e}")
    assert abs(n_or - target) <= 1e-8 + 1e-9


def lapack_frozen_count(s, mu, k, scale):
    """N_k(mu) of Algorithm 1 with the k-step polynomial in place of signum,
    by the independent dense-index route (the pinned route of the oracle tests:
    the submatrix of every group taken from the dense K, eigenpairs by LAPACK),
    with the own-column weights w_l = sum_{c in own} Q_cl^2."""
    import oracle
    kd = s.to_dense()
    boff = block_offsets(s.blk_size)
    stored = np.zeros((s.nblk, s.nblk), dtype=bool)
    for j in range(s.nblk):
        stored[s.row_idx[s.col_ptr[j]:s.col_ptr[j + 1]], j] = True
    tot = 0.0
    for g in range(s.ngroups):
        cols = s.grp_blocks[s.grp_ptr[g]:s.grp_ptr[g + 1]]
        rows = np.nonzero(stored[:, cols].any(axis=1))[0]
        idx = np.concatenate([np.arange(boff[r], boff[r + 1]) for r in rows])
        lam, q = np.linalg.eigh(kd[np.ix_(idx, idx)])
        own = np.searchsorted(idx, np.concatenate([np.arange(boff[j], boff[j + 1]) for j in cols]))
        w = (q[own, :] ** 2).sum(axis=0)
        tot += float((w * 0.5 * (1.0 - oracle.ns_poly((lam - mu) / scale[g], k[g]))).sum())
    return tot


@pytest.mark.timeout(600)
def test_find_mu_water256(smx):
    """The 256-molecule system: mu search to N_e = n/2 within 1e-8 on the
    frozen map.  Pinned by the independent LAPACK route: N_k(mu*) from every
    group's eigenpairs at the search's k_g and s_g.  The search's frozen map is
    also evaluated again at mu*: its slope must be positive and central
    differences of it must match that slope."""
    s = water_config("water256")
    ctx = smx.Context(0).load(s).configure(precision="fp64")
    target = s.n / 2
    mu, steps = smx.smx_find_mu(ctx.handle, target, 1e-8, 60)
    info = ctx.group_info()        # the last evaluation was the frozen one at mu*
    # the search's last evaluation ran the frozen map at mu*: freeze it again
    smx.smx_set_frozen(ctx.handle, True)
    n0, d0 = n_and_slope(smx, ctx, mu)
    h = 1e-5
    fd = (n_and_slope(smx, ctx, mu + h)[0] - n_and_slope(smx, ctx, mu - h)[0]) / (2 * h)
    ctx.close()
    print(f"water256 mu search: mu* = {mu:.10f} in {steps} evaluations; N_k(mu*) - N_e = {n0 - target:.2e}, "
          f"dN/dmu = {d0:.6f} (central difference {fd:.6f})")
    assert d0 > 0
    assert abs(fd - d0) <= 1e-5 * abs(d0)
    assert abs(n0 - target) <= 1e-8 + 1e-9
    n_ref = lapack_frozen_count(s, mu, info["iters"], info["scale"])
    print(f"water256: LAPACK-route N_k(mu*) - N_e = {n_ref - target:.2e}")
    assert abs(n_ref - target) <= 1e-8 + 1e-9
