"""GPU: the debug checks (smx_set_debug_checks) -- host validation of every plan
table and guard regions after the arena, the polish pool and D -- pass on the
path's configurations and leave the results bitwise unchanged: FP64, 2-word
FP16 on 128 x 128 and 256 x 256 tiles, several waves, the diagonalisation path
and the element-level split problem."""

import numpy as np
import pytest

from waterbox import water_config, random_block_system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smx():
    import paper_2004_10811_amd as smx
    smx.load_library()
    return smx


def ragged():
    return random_block_system(61, [13, 5, 5, 17, 9, 31, 22, 13, 27, 11, 5, 25] * 2, density=0.45,
                               coupling=0.02, groups="pairs", mu=0.0)


CASES = {
    "water16-fp64": lambda smx: (water_config("water16"), dict(precision="fp64"), None),
    "ragged-fp16x2-128": lambda smx: (ragged(), dict(precision="fp16x2", tile_shape=0), None),
    "ragged-fp16x2-256": lambda smx: (ragged(), dict(precision="fp16x2", tile_shape=32), None),
    "ragged-fp64-waves": lambda smx: (ragged(), dict(precision="fp64", workspace_limit=8 << 20), None),
    "water16-eig": lambda smx: (water_config("water16"), dict(precision="fp64", kT=0.01), None),
    "water16e-split": lambda smx: (None, dict(precision="fp64"), smx.split_columns(water_config("water16e"), 1e-5)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_debug_checks_pass_and_change_nothing(smx, case):
    s, cfg, sp = CASES[case](smx)
    prob = sp if sp is not None else s
    out = []
    for dbg in (False, True):
        ctx = smx.Context(0).load(prob).configure(**cfg)
        smx.smx_set_debug_checks(ctx.handle, dbg)
        r = ctx.evaluate()
        out.append((r.d_values.copy(), r.n_elec, r.energy, ctx.stats()["nwaves"]))
        ctx.close()
    print(f"{case}: {out[0][3]} wave(s), N = {out[0][1]:.6f}")
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1] and out[0][2] == out[1][2]
