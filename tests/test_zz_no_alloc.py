"""GPU: smx_evaluate_static, the evaluation that allocates nothing.

All of its work memory comes from one fixed device array inside the library,
shared by every call on the device, so each call must clear what it reads
before writing it.  Checked here against smx_evaluate on the same inputs
(bitwise, which implies the 1e-10 / 1e-6 parity bars): two static calls in a
row, the second on a smaller problem; a problem that needs several waves of
the array; switching between the two entry points on one context; and the
error for a group too large for the array.
"""

import numpy as np
import pytest

from waterbox import water_config, random_block_system

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp16x2": 1e-6, "bf16x3": 1e-6, "fp32": 1e-6}


@pytest.fixture(scope="module")
def smx():
    import paper_2004_10811_amd as smx
    smx.load_library()
    return smx


def _pair(smx, s, precision):
    """smx_evaluate and then smx_evaluate_static on one context."""
    ctx = smx.Context(0).load(s).configure(precision=precision)
    ref = ctx.evaluate()
    ref_d = ref.d_values.copy()
    got = ctx.evaluate_static()
    out = (ref_d, ref.n_elec, ref.energy, ref.status, got.d_values.copy(), got.n_elec, got.energy, got.status)
    ctx.close()
    return out


def _check(precision, name, out):
    ref_d, ref_n, ref_e, ref_st, d, n, e, st = out
    err = float(np.abs(d - ref_d).max())
    print(f"{name} {precision}: static vs smx_evaluate max|dD| = {err:.1e}, N {n:.10f} / {ref_n:.10f}")
    assert st == ref_st
    assert err <= TOL[precision]
    assert np.array_equal(d, ref_d) and n == ref_n and e == ref_e


@pytest.mark.parametrize("precision", ["fp64", "fp16x2"])
def test_two_calls_second_smaller(smx, precision):
    # water256 needs several waves of the fixed array in either mode
    big = water_config("water256")
    small = random_block_system(73, [13, 5, 5, 17, 9, 31, 22, 13, 27, 11, 5, 25], density=0.45,
                                coupling=0.05, groups="pairs", mu=0.01)
    _check(precision, "water256", _pair(smx, big, precision))
    _check(precision, "ragged", _pair(smx, small, precision))


@pytest.mark.parametrize("precision", ["fp64", "fp16x2", "bf16x3", "fp32"])
def test_water16_all_modes(smx, precision):
    _check(precision, "water16", _pair(smx, water_config("water16"), precision))


def test_entry_points_interleaved(smx):
    """static, library-arena, static again on one context, after another
    context's static call has overwritten the array."""
    s = water_config("water16")
    other = random_block_system(75, [13, 5, 5, 17, 9, 31], density=0.5, coupling=0.05, groups="pairs", mu=0.0)
    ctx = smx.Context(0).load(s).configure(precision="fp16x2")
    a = ctx.evaluate_static()
    da = a.d_values.copy()
    b = ctx.evaluate()
    db = b.d_values.copy()
    ctx2 = smx.Context(0).load(other).configure(precision="fp64")
    ctx2.evaluate_static()
    ctx2.close()
    c = ctx.evaluate_static()
    dc = c.d_values.copy()
    with pytest.raises(smx.SmxError) as ei:
        ctx.stats()
    assert ei.value.code == smx.SMX_E_STATE
    ctx.close()
    assert np.array_equal(da, db) and np.array_equal(dc, db)
    assert a.n_elec == b.n_elec == c.n_elec and a.energy == b.energy == c.energy


def test_group_too_large_for_the_array(smx):
    # one dense group of n = 6500: 26 n_pad^2 bytes of iterates alone exceed 1 GiB
    s = random_block_system(77, [500] * 13, density=1.0, coupling=0.01, groups="all", mu=0.0)
    ctx = smx.Context(0).load(s).configure(precision="fp16x2")
    with pytest.raises(smx.SmxError) as ei:
        ctx.evaluate_static()
    ctx.close()
    print(ei.value)
    assert ei.value.code == smx.SMX_E_NOMEM
