"""Waves: groups processed in consecutive batches that share one work arena.

A work-space limit forces several waves on small systems; every group's
arithmetic is independent of the wave it falls in, so D, N, E, the per-group
step counts and residuals must equal the single-wave run bit for bit, and
still match the FP64 oracle.
"""

import numpy as np
import pytest

from waterbox import water_config, random_block_system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smx():
    import paper_2004_10811_amd as smx
    smx.load_library()
    return smx


def group_bytes(n, m_own):
    """Work space one group adds to a wave (26 B per slab element + own-column blocks)."""
    npad = -(-n // 32) * 32
    return 26 * npad * npad + 72 * npad * m_own


def own_widths(s):
    widths = []
    for g in range(s.ngroups):
        cols = s.grp_blocks[s.grp_ptr[g]:s.grp_ptr[g + 1]]
        widths.append(int(sum(s.blk_size[j] for j in cols)))
    return np.array(widths)


def run(smx, s, precision, limit=0):
    ctx = smx.Context(0).load(s)
    ctx.configure(precision=precision, workspace_limit=limit)
    res = ctx.evaluate()
    info = ctx.group_info()
    stats = ctx.stats()
    ctx.close()
    return res, info, stats


def forcing_limit(s, info, per_wave=3):
    b = [group_bytes(int(n), int(m)) for n, m in zip(info["n"], own_widths(s))]
    return per_wave * max(b)


@pytest.mark.parametrize("precision", ["fp64", "fp16x2", "bf16x3"])
def test_waves_bitwise_equal_single_wave(smx, oracle_lib, precision):
    s = water_config("water16")
    r1, i1, s1 = run(smx, s, precision)
    assert s1["nwaves"] == 1
    limit = forcing_limit(s, i1)
    rw, iw, sw = run(smx, s, precision, limit)
    print(f"water16 {precision}: {sw['nwaves']} waves under {limit} bytes")
    assert sw["nwaves"] >= 4
    np.testing.assert_array_equal(rw.d_values, r1.d_values)
    assert rw.n_elec == r1.n_elec and rw.energy == r1.energy
    np.testing.assert_array_equal(iw["iters"], i1["iters"])
    np.testing.assert_array_equal(iw["resid"], i1["resid"])
    np.testing.assert_array_equal(iw["scale"], i1["scale"])
    ref = oracle_lib.submatrix(s)
    ok = ~np.isnan(ref.d_values)
    tol = 1e-10 if precision == "fp64" else 1e-6
    assert float(np.abs(rw.d_values[ok] - ref.d_values[ok]).max()) <= tol


def test_waves_uneven_groups_match_oracle(smx, oracle_lib):
    """Ragged block sizes, combined block columns, one wave per group."""
    s = random_block_system(14, [17, 9, 31, 4, 22, 13, 8, 27, 19, 11, 6, 25, 14], density=0.6,
                            coupling=0.04, groups="pairs", mu=0.01)
    r1, i1, _ = run(smx, s, "fp64")
    rw, _, sw = run(smx, s, "fp64", forcing_limit(s, i1, per_wave=1))
    assert sw["nwaves"] == s.ngroups
    np.testing.assert_array_equal(rw.d_values, r1.d_values)
    ref = oracle_lib.submatrix(s)
    assert float(np.abs(rw.d_values - ref.d_values).max()) <= 1e-10


def test_waves_mu_search_and_tangent(smx):
    s = water_config("water16")
    r1, i1, _ = run(smx, s, "fp64")
    limit = forcing_limit(s, i1)
    mus = []
    for lim in (0, limit):
        ctx = smx.Context(0).load(s).configure(precision="fp64", workspace_limit=lim)
        mus.append(smx.smx_find_mu(ctx.handle, round(r1.n_elec) + 0.5, 1e-8, 30))
        ctx.close()
    assert mus[0][0] == mus[1][0] and mus[0][1] == mus[1][1]


def test_waves_limits_of_the_api(smx):
    s = water_config("water16")
    r1, i1, _ = run(smx, s, "fp64")
    ctx = smx.Context(0).load(s).configure(precision="fp64", workspace_limit=forcing_limit(s, i1))
    ctx.evaluate()
    assert ctx.stats()["nwaves"] >= 4
    # the last wave's iterates are kept; earlier waves' were overwritten
    last = s.ngroups - 1
    x = ctx.submatrix(last, what=1)
    assert np.all(np.isfinite(x))
    with pytest.raises(smx.SmxError) as e:
        ctx.submatrix(0, what=1)
    assert e.value.code == smx.SMX_E_UNSUPPORTED
    # the gathered A_g (what = 0) is served for any group
    a0 = ctx.submatrix(0, what=0)
    assert a0.shape[0] == i1["n"][0]
    with pytest.raises(smx.SmxError) as e:
        ctx.backward(1.0, 0.0)
    assert e.value.code == smx.SMX_E_UNSUPPORTED
    # a limit below one group's need is refused when the plan is built
    smx.smx_set_workspace_limit(ctx.handle, 1 << 16)
    with pytest.raises(smx.SmxError) as e:
        smx.smx_evaluate(ctx.handle)
    assert e.value.code == smx.SMX_E_NOMEM
    ctx.close()


@pytest.mark.timeout(900)
def test_water6912_mixed_in_waves_sampled_groups(smx, oracle_lib):
    """6912 molecules (158,976 basis functions): the slabs exceed one GPU's
    memory, so the groups run in waves; sampled groups (largest, smallest,
    and seeded random ones from different waves) match the oracle."""
    s = water_config("water6912")
    print(f"water6912 generated: {s.n} basis functions", flush=True)
    ctx = smx.Context(0).load(s).configure(precision="fp16x2")
    res = ctx.evaluate()
    info = ctx.group_info()
    stats = ctx.stats()
    ctx.close()
    print(f"water6912 evaluated in {stats['nwaves']} waves", flush=True)
    n_g = info["n"]
    rng = np.random.default_rng(6912)
    pick = {int(np.argmax(n_g)), int(np.argmin(n_g)), 0, s.ngroups - 1}
    while len(pick) < 6:
        pick.add(int(rng.integers(s.ngroups)))
    ref = oracle_lib.submatrix(s, which=sorted(pick), nthreads=6)
    ok = ~np.isnan(ref.d_values)
    err = float(np.abs(res.d_values[ok] - ref.d_values[ok]).max())
    print(f"water6912 fp16x2: {stats['nwaves']} waves, n_g {stats['n_min']}-{stats['n_max']}, "
          f"sampled {sorted(pick)}: max|dD| = {err:.2e}; {stats['time_total_ms']:.0f} ms")
    assert stats["nwaves"] >= 2
    assert stats["n_not_converged"] == 0
    assert err <= 1e-6
    assert np.all(np.isfinite(res.d_values))
