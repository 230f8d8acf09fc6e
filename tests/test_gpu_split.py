"""GPU: the sub-submatrix method (Sec. IV-C, "Splitting up submatrices") against
the oracle.

smx_split_columns builds the element-level problem (one sub-submatrix per
column, rows where the column is non-zero above the element cutoff), the
ordinary GPU path evaluates it, and smx_get_d_expanded writes D back in K's
block layout.  D must match the oracle's split method element by element
(1e-10 FP64, 1e-6 2-word FP16); with no cutoff the split must reproduce the
block-column submatrices bit for bit; and the water256e case reports the time against the block-level
groups beside the work ratio sum n^3 of Eq. estimatedspeedup.
"""

import numpy as np
import pytest

from waterbox import water_config

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp16x2": 1e-6}
EPS = 1e-5


@pytest.fixture(scope="module")
def smx():
    import paper_2004_10811_amd as smx
    smx.load_library()
    return smx


def run_split(smx, s, precision, merge=True):
    sp = smx.split_columns(s, EPS, merge=merge)
    ctx = smx.Context(0).load(sp).configure(precision=precision)
    r = ctx.evaluate()
    d = smx.smx_get_d_expanded(ctx.handle, sp.src, len(s.values))
    out = dict(d=d, n=r.n_elec, e=r.energy, ms=ctx.stats()["time_total_ms"], sp=sp,
               work=smx.group_speedup(sp)[1])
    ctx.close()
    return out


@pytest.fixture(scope="module")
def water16e_ref(oracle_lib):
    s = water_config("water16e")
    return s, oracle_lib.split_submatrix(s, EPS)


@pytest.mark.parametrize("precision", ["fp64", "fp16x2"])
def test_water16e_matches_oracle(smx, water16e_ref, precision):
    s, ref = water16e_ref
    r = run_split(smx, s, precision)
    err = float(np.abs(r["d"] - ref.d_values).max())
    print(f"water16e {precision}: {len(r['sp'].grp_ptr) - 1} sub-submatrices, max|dD| = {err:.2e}, "
          f"dN = {r['n'] - ref.n_elec:.1e}, dE = {r['e'] - ref.energy:.1e}, {r['ms']:.2f} ms")
    assert err <= TOL[precision]
    assert abs(r["n"] - ref.n_elec) <= TOL[precision] * s.n
    assert abs(r["e"] - ref.energy) <= TOL[precision] * s.n


def test_no_cutoff_equals_block_columns_bitwise(smx):
    """eps = 0 on water16 (no zero elements): every column of a block column keeps
    the rows of its block column's submatrix, so the merged groups are the block
    columns and D is bitwise the block-level result with single-block-column
    groups; single-column groups solve the same matrices again."""
    s = water_config("water16")
    cols = s.with_groups([[j] for j in range(s.nblk)])
    ctx = smx.Context(0).load(cols).configure(precision="fp64")
    ref = ctx.evaluate()
    d_ref = ref.d_values.copy()
    ctx.close()
    for merge in (True, False):
        sp = smx.split_columns(s, 0.0, merge=merge)
        assert (len(sp.grp_ptr) - 1) == (s.nblk if merge else s.n)
        ctx = smx.Context(0).load(sp).configure(precision="fp64")
        r = ctx.evaluate()
        d = smx.smx_get_d_expanded(ctx.handle, sp.src, len(s.values))
        ctx.close()
        assert np.array_equal(d, d_ref)
        assert abs(r.n_elec - ref.n_elec) <= 1e-11 and abs(r.energy - ref.energy) <= 1e-11


def test_expand_refuses_bad_index(smx):
    s = water_config("water16e")
    sp = smx.split_columns(s, EPS)
    ctx = smx.Context(0).load(sp).configure(precision="fp64")
    ctx.evaluate()
    bad = sp.src.copy()
    bad[5] = bad[6]
    for idx, n_out in ((bad, len(s.values)), (sp.src, int(sp.src.max()))):
        with pytest.raises(smx.SmxError) as ei:
            smx.smx_get_d_expanded(ctx.handle, idx, n_out)
        assert ei.value.code == smx.SMX_E_INVALID
    ctx.close()


def test_water256e_sampled_and_timed(smx, oracle_lib):
    s = water_config("water256e")
    r = run_split(smx, s, "fp16x2")
    ctx = smx.Context(0).load(s).configure(precision="fp16x2")
    ctx.evaluate()
    ms_blk = ctx.stats()["time_total_ms"]
    ctx.close()
    work_blk = smx.group_speedup(s)[1]
    rng = np.random.default_rng(8)
    pick = sorted({int(x) for x in rng.integers(s.ngroups, size=3)})
    ref = oracle_lib.split_submatrix(s, EPS, which=pick)
    ok = ~np.isnan(ref.d_values)
    err = float(np.abs(r["d"][ok] - ref.d_values[ok]).max())
    print(f"water256e fp16x2: split {len(r['sp'].grp_ptr) - 1} sub-submatrices {r['ms']:.2f} ms, "
          f"molecule groups {ms_blk:.2f} ms; sum n^3 ratio (molecules / split) {work_blk / r['work']:.3f}; "
          f"max|dD| vs oracle on groups {pick} = {err:.2e}")
    assert err <= TOL["fp16x2"]


def test_split_at_finite_temperature(smx, oracle_lib):
    """The split problem through the diagonalisation path (kT = 0.05): the oracle's
    split method with the Fermi function, element by element."""
    s = water_config("water16e")
    kT = 0.05
    ref = oracle_lib.split_submatrix(s, EPS, kT=kT)
    sp = smx.split_columns(s, EPS, merge=True)
    ctx = smx.Context(0).load(sp).configure(precision="fp64", kT=kT)
    r = ctx.evaluate()
    d = smx.smx_get_d_expanded(ctx.handle, sp.src, len(s.values))
    ctx.close()
    err = float(np.abs(d - ref.d_values).max())
    print(f"water16e split kT = {kT}: max|dD| = {err:.2e}, dN = {r.n_elec - ref.n_elec:.1e}")
    assert err <= TOL["fp64"]
    assert abs(r.n_elec - ref.n_elec) <= 1e-9 and abs(r.energy - ref.energy) <= 1e-9
