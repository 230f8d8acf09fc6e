"""GPU parity of the reduced-precision paths against the FP64 CPU oracle.

Bar: max|D_gpu - D_oracle| <= 1e-6 for the modes meant to meet it (2-word
FP16, 3-word BF16 and FP32 bulk, FP64 polish).  The tolerance follows from the
arithmetic: FP32 accumulation of exact word products injects ~1e-7 relative
noise per product; the occupied-virtual part of that noise is not removed by
later steps (it is amplified by up to 1.5 per step while the eigenvalues near
mu are small), and CPU simulations of 16 water1024 submatrices put the final
error at 3-7e-7.  The single-word BF16 mode is the literal low-precision run;
its error (~1e-3) is reported, and only loosely bounded here.
"""

import numpy as np
import pytest

from waterbox import water_config, random_block_system

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-6


@pytest.fixture(scope="module")
def smx():
    import paper_2004_10811_amd as smx
    smx.load_library()
    return smx


def run(smx, s, precision, allow_not_converged=False, **kw):
    ctx = smx.Context(0).load(s)
    ctx.configure(precision=precision, **kw)
    res = ctx.evaluate(allow_not_converged=allow_not_converged)
    info = ctx.group_info()
    stats = ctx.stats()
    ctx.close()
    return res, info, stats


def max_err(res, ref):
    ok = ~np.isnan(ref.d_values)
    return float(np.abs(res.d_values[ok] - ref.d_values[ok]).max())


@pytest.mark.parametrize("precision", ["fp16x2", "bf16x3", "fp32"])
def test_water16_mixed_matches_oracle(smx, oracle_lib, precision):
    s = water_config("water16")
    res, info, stats = run(smx, s, precision)
    ref = oracle_lib.submatrix(s)
    err = max_err(res, ref)
    print(f"water16 {precision}: max|dD| = {err:.2e}, dN = {res.n_elec - ref.n_elec:.2e}, "
          f"dE = {res.energy - ref.energy:.2e}, steps {stats['iters_min']}-{stats['iters_max']}")
    assert err <= TOL_MIXED
    assert abs(res.n_elec - ref.n_elec) <= TOL_MIXED * s.n
    assert stats["n_not_converged"] == 0
    # residual of the last full FP64 iterate on the own columns: one quadratic
    # step from the bulk switch (<= 1e-3) leaves ~1e-6; the final own-column
    # step squares it again
    assert np.all(info["resid"] <= 1e-5)


def test_water16_bf16_single_word_is_reported(smx, oracle_lib):
    """Literal low-precision run (BF16 words, FP32 accumulation, 2 FP64 polish steps).

    Its bulk stalls at the BF16 rounding floor (tau ~ 1e-2, accepted for this
    mode), and two FP64 polish steps from there leave the returned iterate's
    residual above tol = 1e-12, so the call reports SMX_E_NOT_CONVERGED with D
    written; with a third polish step the iteration converges.  Either way D
    is the sign of the rounded bulk iterate, ~1e-3 from the oracle (reported)."""
    s = water_config("water16")
    res, info, stats = run(smx, s, "bf16", allow_not_converged=True)
    ref = oracle_lib.submatrix(s)
    err = max_err(res, ref)
    print(f"water16 bf16 (1 word): status {res.status}, max|dD| = {err:.2e}, dN = {res.n_elec - ref.n_elec:.2e}, "
          f"dE = {res.energy - ref.energy:.2e}, steps {stats['iters_min']}-{stats['iters_max']}, "
          f"polished residual max {info['resid'].max():.2e}")
    assert err < 2e-2
    assert np.all(np.isfinite(res.d_values))
    assert res.status in (smx.SMX_OK, smx.SMX_E_NOT_CONVERGED)
    # the flag agrees with the documented rule on the polished residual
    expect_nc = int(np.sum(0.75 * info["resid"] ** 2 > 1e-12))
    assert stats["n_not_converged"] == expect_nc
    assert (res.status == smx.SMX_E_NOT_CONVERGED) == (expect_nc > 0)
    res4, info4, stats4 = run(smx, s, "bf16", allow_not_converged=True, n_polish=4)
    print(f"water16 bf16 (1 word), 4 polish steps: status {res4.status}, max|dD| = {max_err(res4, ref):.2e}, "
          f"polished residual max {info4['resid'].max():.2e}")
    assert res4.status == smx.SMX_OK and stats4["n_not_converged"] == 0


@pytest.mark.parametrize("seed,sizes,dens,groups", [
    (11, [3, 1, 7, 2, 5, 4, 6, 1, 8, 3, 2, 5], 0.35, "column"),
    (12, [13, 5, 5] * 6, 0.5, "pairs"),
    (14, [17, 9, 31, 4, 22, 13, 8, 27, 19, 11, 6, 25, 14], 0.6, "all"),
])
def test_random_systems_mixed(smx, oracle_lib, seed, sizes, dens, groups):
    s = random_block_system(seed, sizes, density=dens, coupling=0.04, groups=groups, mu=0.01)
    ref = oracle_lib.submatrix(s)
    for precision in ("fp16x2", "bf16x3", "fp32"):
        res, _, _ = run(smx, s, precision)
        assert max_err(res, ref) <= TOL_MIXED, precision


@pytest.mark.parametrize("precision", ["fp16x2", "bf16x3", "bf16", "fp32"])
def test_bulk_iterate_readback_matches_oracle_sign(smx, oracle_lib, precision):
    """smx_get_submatrix(what = 1) in the reduced modes converts the bulk's last
    iterate from its word storage to FP64.  That iterate stops at tau_k =
    Tr(I - X_k^2) <= 1e-3 (or the word floor), so every eigenvalue is within
    tau_k / 2 of +-1 and the entries are within about tau_k of the exact sign
    Q signum(Lambda) Q^T of the oracle's eigendecomposition; the 1-word BF16
    run stalls at its floor (~1e-2)."""
    s = water_config("water16")
    ctx = smx.Context(0).load(s).configure(precision=precision)
    ctx.evaluate(allow_not_converged=(precision == "bf16"))
    tol = 2e-2 if precision == "bf16" else 2e-3
    for g in (0, s.ngroups // 2, s.ngroups - 1):
        x = ctx.submatrix(g, what=1)
        _, lam, q, _ = oracle_lib.group_eig(s, g)
        sign = (q * np.sign(lam)) @ q.T
        assert x.shape == sign.shape
        err = float(np.abs(x - sign).max())
        print(f"water16 {precision} group {g}: max|X_bulk - sign| = {err:.2e}")
        assert err <= tol, (g, err)
        # symmetric to the word rounding
        assert float(np.abs(x - x.T).max()) <= 1e-5
        # re-gathering A_g (what = 0) leaves the stored iterates alone
        a = ctx.submatrix(g, what=0)
        assert a.shape == x.shape
        np.testing.assert_array_equal(ctx.submatrix(g, what=1), x)
    ctx.close()


def test_mixed_polish_count_and_determinism(smx, oracle_lib):
    s = water_config("water16")
    ctx = smx.Context(0).load(s).configure(precision="fp16x2", n_polish=3)
    a = ctx.evaluate()
    b = ctx.evaluate()
    st = ctx.stats()
    ctx.close()
    np.testing.assert_array_equal(a.d_values, b.d_values)
    ref = oracle_lib.submatrix(s)
    assert max_err(a, ref) <= TOL_MIXED
    res_fp64, _, st64 = run(smx, s, "fp64")
    # same number of steps to within a couple (bulk + 3 polish vs FP64 to 1e-12)
    assert abs(st["iters_mean"] - st64["iters_mean"]) < 3


@pytest.mark.timeout(600)
def test_water1024_mixed_sampled_groups(smx, oracle_lib):
    """Full-size 1024-molecule system in the benchmark's launch configuration."""
    s = water_config("water1024")
    res, info, stats = run(smx, s, "fp16x2")
    n_g = info["n"]
    rng = np.random.default_rng(4321)
    pick = {int(np.argmax(n_g)), int(np.argmin(n_g))}
    while len(pick) < 6:
        pick.add(int(rng.integers(s.ngroups)))
    ref = oracle_lib.submatrix(s, which=sorted(pick))
    err = max_err(res, ref)
    print(f"water1024 fp16x2 sampled {sorted(pick)}: max|dD| = {err:.2e}; steps "
          f"{stats['iters_min']}-{stats['iters_max']}; {stats['time_total_ms']:.1f} ms")
    assert err <= TOL_MIXED
    assert stats["n_not_converged"] == 0


def _edge_gap_system(oracle_lib, seed, sizes, gap):
    """Ragged random system with mu placed `gap` above the highest occupied
    submatrix eigenvalue (over all groups), so min over groups of |lambda - mu|
    equals `gap` exactly (test-only use of the oracle's eigendecompositions).
    Couplings of 0.02 keep the union of the group spectra gapped around 0
    (occupied <= -0.24, virtual >= +0.27 for seed 31), so no virtual
    eigenvalue comes closer to mu than `gap`."""
    s = random_block_system(seed, sizes, density=0.45, coupling=0.02, groups="pairs", mu=0.0)
    top = -np.inf
    for g in range(s.ngroups):
        _, lam, _, _ = oracle_lib.group_eig(s, g, mu=0.0)
        occ = lam[lam < 0]
        if occ.size:
            top = max(top, float(occ.max()))
    mu = top + gap
    mind = np.inf
    for g in range(s.ngroups):
        _, lam, _, _ = oracle_lib.group_eig(s, g, mu=mu)
        mind = min(mind, float(np.abs(lam).min()))
    assert 0.5 * gap <= mind <= gap * (1 + 1e-9) + 1e-15
    return s, mu, mind


@pytest.mark.parametrize("gap", [1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6])
@pytest.mark.parametrize("precision", ["fp16x2", "bf16x3", "fp32"])
def test_small_gap_meets_bar_or_flags(smx, oracle_lib, precision, gap):
    """min|lambda - mu| from 1e-1 down to 1e-6 on ragged systems (several tiles
    and ragged tails): every group either meets max|dD| <= 1e-6 against the
    oracle, or the call reports SMX_E_NOT_CONVERGED; a converged status with a
    larger error would be a silent failure."""
    s, mu, mind = _edge_gap_system(oracle_lib, 31, [13, 5, 5, 17, 9, 31, 22, 13, 27, 11, 5, 25] * 2, gap)
    ref = oracle_lib.submatrix(s, mu=mu)
    res, info, stats = run(smx, s, precision, allow_not_converged=True, mu=mu)
    err = max_err(res, ref)
    r64, _, st64 = run(smx, s, "fp64", mu=mu)
    print(f"gap {mind:.2e} {precision}: status {res.status}, max|dD| = {err:.2e}, "
          f"not converged {stats['n_not_converged']}/{s.ngroups}, steps {stats['iters_min']}-{stats['iters_max']} "
          f"(FP64 {st64['iters_min']}-{st64['iters_max']}, max|dD| {max_err(r64, ref):.1e})")
    assert max_err(r64, ref) <= 1e-10
    assert np.all(np.isfinite(res.d_values))
    if res.status == smx.SMX_OK:
        assert err <= TOL_MIXED
    else:
        assert res.status == smx.SMX_E_NOT_CONVERGED and stats["n_not_converged"] > 0


@pytest.mark.parametrize("precision", ["fp16x2", "bf16x3", "fp32"])
def test_step_cap_reports_not_converged(smx, precision):
    """A bulk cut off by max_iter (here n_polish + 3 steps) leaves tau far above
    switch_tol: the call must say so, with D still written."""
    s = water_config("water16")
    res, info, stats = run(smx, s, precision, allow_not_converged=True, max_iter=5, n_polish=2)
    assert res.status == smx.SMX_E_NOT_CONVERGED
    assert stats["n_not_converged"] == s.ngroups
    assert np.all(np.isfinite(res.d_values))


@pytest.mark.parametrize("precision", ["fp64", "fp16x2", "fp32"])
def test_small_scale_prescaling_keeps_padding_fixed(smx, oracle_lib, precision):
    """K scaled by 0.2 gives Gershgorin scales s_g < 0.447: a padded diagonal
    entry prescaled like the true block (1/s_g > sqrt(5)) would diverge under
    x (3 - x^2) / 2.  Ragged sizes make every group carry padding."""
    base = random_block_system(41, [13, 5, 5, 7, 3, 11, 9, 5, 13, 6], density=0.5, coupling=0.04,
                               groups="pairs", mu=0.0)
    s = base.with_values(base.values * 0.2)
    ref = oracle_lib.submatrix(s)
    res, info, stats = run(smx, s, precision)
    print(f"scaled K {precision}: s_g {info['scale'].min():.3f}-{info['scale'].max():.3f}, "
          f"max|dD| = {max_err(res, ref):.2e}")
    assert info["scale"].max() < 0.447
    assert np.all(info["n"] % 32 != 0)
    assert max_err(res, ref) <= (1e-10 if precision == "fp64" else TOL_MIXED)
