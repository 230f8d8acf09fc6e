"""GPU: submatrices built from k-means groups of block columns (Sec. IV-C).

The grouping changes which submatrices are solved, not what D means: the GPU
path on k-means groups of water256 must match the oracle on the same groups
(sampled), and the measured time of the sign step should follow the work
sum_g n_g^3 that Eq. estimatedspeedup compares (printed; the bar is on D).
"""

import numpy as np
import pytest

from waterbox import water_config

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp16x2": 1e-6}


@pytest.fixture(scope="module")
def smx():
    import paper_2004_10811_amd as smx
    smx.load_library()
    return smx


def regroup(s, gp, gb):
    return s.with_groups([list(gb[gp[g]:gp[g + 1]]) for g in range(len(gp) - 1)])


@pytest.mark.parametrize("precision", ["fp64", "fp16x2"])
def test_kmeans_groups_match_oracle(smx, oracle_lib, precision):
    base = water_config("water256")
    box = base.meta["box"]
    gp, gb = smx.group_kmeans(base.coords, 384, box=box, seed=3)
    s = regroup(base, gp, gb)
    sp, work = smx.group_speedup(s)
    ctx = smx.Context(0).load(s).configure(precision=precision)
    r = ctx.evaluate()
    d = r.d_values.copy()
    ms = ctx.stats()["time_total_ms"]
    ctx.close()
    ctx = smx.Context(0).load(base).configure(precision=precision)
    ctx.evaluate()
    ms_mol = ctx.stats()["time_total_ms"]
    ctx.close()
    rng = np.random.default_rng(5)
    pick = sorted({int(x) for x in rng.integers(s.ngroups, size=3)})
    ref = oracle_lib.submatrix(s, which=pick)
    ok = ~np.isnan(ref.d_values)
    err = float(np.abs(d[ok] - ref.d_values[ok]).max())
    print(f"water256 {precision}: {s.ngroups} k-means groups, S vs molecules "
          f"{smx.group_speedup(base)[1] / work:.3f}, {ms:.2f} ms (molecules {ms_mol:.2f} ms); "
          f"max|dD| on {pick} = {err:.2e}")
    assert err <= TOL[precision]


@pytest.mark.parametrize("kT", [0.0, 0.02])
def test_kmeans_groups_diagonalisation(smx, oracle_lib, kT):
    """k-means groups of water16 (8 clusters) through the diagonalisation path
    against the oracle on every group."""
    base = water_config("water16")
    gp, gb = smx.group_kmeans(base.coords, 8, box=base.meta["box"], seed=4)
    s = regroup(base, gp, gb)
    ref = oracle_lib.submatrix(s, kT=kT)
    ctx = smx.Context(0).load(s).configure(precision="fp64", kT=kT, solver="eig")
    r = ctx.evaluate()
    ctx.close()
    err = float(np.abs(r.d_values - ref.d_values).max())
    print(f"water16 k-means 8 groups, kT = {kT}: max|dD| = {err:.2e}")
    assert err <= TOL["fp64"]
    assert abs(r.n_elec - ref.n_elec) <= 1e-9
