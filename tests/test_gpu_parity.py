"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bar (FP64 path): max|D_gpu - D_oracle| <= 1e-10 element by element, and the
same for N = Tr D and E = Tr(DK) scaled by their size.  The tolerance: the
Newton-Schulz iterate stops at max|X^2 - I| <= 1e-12, which bounds its
distance to the exact sign by the same order; FP64 rounding in products of
dimension n <= ~1000 adds ~n u ~ 1e-13; the oracle's Jacobi is accurate to
~1e-14.  1e-10 leaves two orders of margin.
"""

import numpy as np
import pytest

from waterbox import water_config, water_system, random_block_system, tb_chain

pytestmark = pytest.mark.gpu

TOL_D = 1e-10


@pytest.fixture(scope="module")
def smx():
    import paper_2004_10811_amd as smx
    smx.load_library()
    return smx


def run_gpu(smx, s, precision="fp64", **kw):
    ctx = smx.Context(0).load(s)
    ctx.configure(precision=precision, **kw)
    res = ctx.evaluate()
    info = ctx.group_info()
    stats = ctx.stats()
    ctx.close()
    return res, info, stats


def compare(s, res, ref, tol=TOL_D):
    ok = ~np.isnan(ref.d_values)
    err = np.abs(res.d_values[ok] - ref.d_values[ok]).max()
    assert err <= tol, f"max|dD| = {err:.3e} > {tol:.1e}"
    return err


def test_water16_fp64_matches_oracle(smx, oracle_lib):
    s = water_config("water16")
    res, info, stats = run_gpu(smx, s)
    ref = oracle_lib.submatrix(s)
    err = compare(s, res, ref)
    assert abs(res.n_elec - ref.n_elec) <= 1e-10 * s.n
    assert abs(res.energy - ref.energy) <= 1e-10 * s.n
    assert stats["n_not_converged"] == 0
    assert np.all(info["resid"] <= 1e-12)
    n_or, _ = oracle_lib.group_dims(s)
    assert np.array_equal(info["n"], n_or)
    print(f"water16 fp64: max|dD| = {err:.2e}, iters {info['iters'].min()}-{info['iters'].max()}")


@pytest.mark.parametrize("case", [
    # (seed, block sizes, density, groups)
    (1, [3, 1, 7, 2, 5, 4, 6, 1, 8, 3, 2, 5], 0.35, "column"),
    (2, [13, 5, 5] * 6, 0.5, "pairs"),
    (3, [1] * 40, 0.2, "column"),
    (4, [17, 9, 31, 4, 22, 13, 8, 27, 19, 11, 6, 25, 14], 0.6, "all"),   # one group, n = 206
    (5, [29, 31, 30, 28, 33, 32, 27, 26, 30, 31], 0.9, "all"),           # n = 297, 3 tiles, ragged
    (6, [64] * 5, 1.0, "column"),                                         # n = 320 = 10 * 32 exactly
])
def test_random_systems_match_oracle(smx, oracle_lib, case):
    seed, sizes, dens, groups = case
    s = random_block_system(seed, sizes, density=dens, coupling=0.04, groups=groups, mu=0.01)
    res, info, stats = run_gpu(smx, s)
    ref = oracle_lib.submatrix(s)
    compare(s, res, ref)
    assert abs(res.n_elec - ref.n_elec) <= 1e-10 * s.n
    assert abs(res.energy - ref.energy) <= 1e-10 * s.n


def test_band_chain_closed_form_on_gpu(smx, oracle_lib):
    s = tb_chain(48, 4, 0.0, -1.0, pattern="band", mu=0.1)
    res, _, _ = run_gpu(smx, s)
    ref = oracle_lib.submatrix(s)
    compare(s, res, ref)


def test_diagonal_only_and_single_element_blocks(smx, oracle_lib):
    # every submatrix is one diagonal block; 1x1 blocks give 1x1 submatrices
    rng = np.random.default_rng(8)
    sizes = [1, 2, 1, 5, 1, 3]
    n = sum(sizes)
    kd = np.diag(rng.choice([-0.7, 0.4, 1.3, -2.0], size=n))
    from waterbox import dense_to_bsc
    off = np.cumsum([0] + sizes)
    for b in range(len(sizes)):
        blk = rng.normal(0, 0.05, (sizes[b], sizes[b]))
        kd[off[b]:off[b + 1], off[b]:off[b + 1]] += (blk + blk.T) / 2
    s = dense_to_bsc(kd, sizes, np.eye(len(sizes), dtype=bool), mu=0.05)
    res, info, _ = run_gpu(smx, s)
    ref = oracle_lib.submatrix(s)
    compare(s, res, ref)


def test_mu_shift_and_group_order_invariance(smx, oracle_lib):
    s = water_system(n_mol=12, box=7.0, r_cut=3.5, seed=31)
    s.mu = 0.07
    res1, _, _ = run_gpu(smx, s)
    ref = oracle_lib.submatrix(s)
    compare(s, res1, ref)
    # same groups listed in reverse order: every group computes the same thing
    ng = s.ngroups
    groups = [list(s.grp_blocks[s.grp_ptr[g]:s.grp_ptr[g + 1]]) for g in range(ng)][::-1]
    res2, _, _ = run_gpu(smx, s.with_groups(groups))
    np.testing.assert_array_equal(res1.d_values, res2.d_values)


def test_repeat_evaluations_are_bitwise_identical(smx):
    s = water_config("water16")
    ctx = smx.Context(0).load(s)
    a = ctx.evaluate()
    b = ctx.evaluate()
    ctx.close()
    np.testing.assert_array_equal(a.d_values, b.d_values)
    assert a.n_elec == b.n_elec and a.energy == b.energy


def test_device_resident_values_and_output(smx, oracle_lib):
    torch = pytest.importorskip("torch")
    s = water_system(n_mol=8, box=6.2, r_cut=3.5, seed=32)
    kv = torch.from_numpy(s.values).cuda()
    ctx = smx.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    ctx.load(s, values=kv)
    out = torch.empty_like(kv)
    r = ctx.evaluate(out=out)
    ctx.close()
    ref = oracle_lib.submatrix(s)
    assert np.abs(out.cpu().numpy() - ref.d_values).max() <= TOL_D
    assert abs(r.n_elec - ref.n_elec) <= 1e-10 * s.n


def test_error_paths(smx):
    s = water_system(n_mol=4, box=5.0, r_cut=3.0, seed=33)
    ctx = smx.Context(0)
    # asymmetric values
    bad = s.values.copy()
    voff = s.val_off()
    j = 1
    p = next(q for q in range(s.col_ptr[j], s.col_ptr[j + 1]) if s.row_idx[q] != j)
    bad[voff[p]] += 1e-3
    with pytest.raises(smx.SmxError) as e:
        ctx.load(s, values=bad)
    assert e.value.code == smx.SMX_E_NOT_SYMMETRIC
    # non-finite values
    bad = s.values.copy()
    bad[5] = np.nan
    with pytest.raises(smx.SmxError) as e:
        ctx.load(s, values=bad)
    assert e.value.code == smx.SMX_E_NONFINITE
    # evaluate before a successful load
    with pytest.raises(smx.SmxError) as e:
        smx.smx_evaluate(ctx.handle)
    assert e.value.code == smx.SMX_E_STATE
    ctx.load(s)
    # finite temperature diagonalises in FP64; a reduced-precision mode is refused
    smx.smx_set_temperature(ctx.handle, 0.01)
    smx.smx_set_precision(ctx.handle, smx.SMX_FP16_2W)
    with pytest.raises(smx.SmxError) as e:
        smx.smx_evaluate(ctx.handle)
    assert e.value.code == smx.SMX_E_UNSUPPORTED
    smx.smx_set_precision(ctx.handle, smx.SMX_FP64)
    r = ctx.evaluate()
    assert r.status == smx.SMX_OK and np.all(np.isfinite(r.d_values))
    smx.smx_set_temperature(ctx.handle, 0.0)
    # bad groups
    with pytest.raises(smx.SmxError) as e:
        smx.smx_set_groups(ctx.handle, [0, 2], [0, 0])
    assert e.value.code == smx.SMX_E_INVALID
    # max_iter = 1: not converged, D still written and finite
    smx.smx_set_convergence(ctx.handle, 1e-12, 1, 2, 1e-3)
    r = ctx.evaluate(allow_not_converged=True)
    assert r.status == smx.SMX_E_NOT_CONVERGED
    assert np.all(np.isfinite(r.d_values))
    st = ctx.stats()
    assert st["n_not_converged"] == st["ngroups"]
    ctx.close()


@pytest.mark.timeout(600)
def test_water1024_sampled_groups_match_oracle(smx, oracle_lib):
    """Full-size 1024-molecule system, same launch as the benchmark; the oracle
    recomputes a seeded sample of groups (largest, smallest, four random)."""
    s = water_config("water1024")
    res, info, stats = run_gpu(smx, s)
    n_g = info["n"]
    rng = np.random.default_rng(1234)
    pick = {int(np.argmax(n_g)), int(np.argmin(n_g))}
    while len(pick) < 6:
        pick.add(int(rng.integers(s.ngroups)))
    ref = oracle_lib.submatrix(s, which=sorted(pick))
    err = compare(s, res, ref)
    assert stats["n_not_converged"] == 0
    # whole-matrix properties that hold at any size
    assert abs(res.n_elec - s.n / 2) < 0.05 * s.ngroups
    print(f"water1024 sampled {sorted(pick)}: max|dD| = {err:.2e}; "
          f"iters {stats['iters_min']}-{stats['iters_max']}; time {stats['time_total_ms']:.1f} ms")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp16x2", 1e-6), ("fp32", 1e-6)])
def test_large_single_submatrix_dimerized_chain(smx, precision, tol):
    """One group holding every block column of a dense-pattern K: the submatrix is
    K itself (n = 2600, 21 tile rows, ragged last tile), so D is the exact density
    matrix, here from a dense LAPACK eigendecomposition.  A dimerized chain
    (hoppings -1.0 / -0.6) has the gap [-0.4, 0.4] at mu = 0, so the 1e-6 bar of
    the reduced-precision modes applies."""
    from waterbox import dense_to_bsc
    n, blk = 2600, 26
    h = np.zeros((n, n))
    hop = np.where(np.arange(n - 1) % 2 == 0, -1.0, -0.6)
    h[np.arange(n - 1), np.arange(1, n)] = hop
    h[np.arange(1, n), np.arange(n - 1)] = hop
    nb = n // blk
    s = dense_to_bsc(h, [blk] * nb, np.ones((nb, nb), dtype=bool), groups=[list(range(nb))], mu=0.0)
    lam, q = np.linalg.eigh(h)
    d_exact = q[:, lam < 0] @ q[:, lam < 0].T
    ctx = smx.Context(0).load(s).configure(precision=precision)
    res = ctx.evaluate()
    ctx.close()
    voff = s.val_off()
    err = 0.0
    for j in range(nb):
        for p in range(int(s.col_ptr[j]), int(s.col_ptr[j + 1])):
            i = int(s.row_idx[p])
            blk_ref = d_exact[i * blk:(i + 1) * blk, j * blk:(j + 1) * blk].T.reshape(-1)
            err = max(err, float(np.abs(res.d_values[voff[p]:voff[p + 1]] - blk_ref).max()))
    print(f"dimerized chain n = {n}, {precision}: max|dD| = {err:.2e}, N = {res.n_elec:.10f}")
    assert err <= tol
    assert abs(res.n_elec - n / 2) <= tol * n
