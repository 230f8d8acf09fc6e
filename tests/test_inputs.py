"""The seeded input generator: shapes, symmetry and reproducibility."""

import numpy as np

from waterbox import water_system, water_config, random_block_system, tb_chain


def test_water16_shape_and_symmetry():
    s = water_config("water16")
    assert s.nblk == 48 and s.n == 368 and s.ngroups == 16
    assert set(np.unique(s.blk_size)) == {5, 13}
    kd = s.to_dense()
    assert np.array_equal(kd, kd.T)
    # exactly n/2 on-site energies at -0.5 (noise is 0.05 std, so the sign of the
    # diagonal entry minus the noise is the on-site sign)
    onsite = np.where(np.arange(s.n) % 2 == 0, -0.5, 0.5)
    assert (onsite < 0).sum() == s.n // 2
    assert np.abs(np.diag(kd) - onsite).max() < 0.5
    # every column stores its diagonal block and rows ascend
    for j in range(s.nblk):
        rows = s.row_idx[s.col_ptr[j]:s.col_ptr[j + 1]]
        assert j in rows and np.all(np.diff(rows) > 0)
    # groups are molecules O, H, H
    assert np.array_equal(s.grp_blocks, np.arange(48))
    assert np.array_equal(s.grp_ptr, np.arange(0, 49, 3))


def test_water_reproducible_and_seed_dependent():
    a = water_system(12, 7.0, 4.0, seed=7)
    b = water_system(12, 7.0, 4.0, seed=7)
    c = water_system(12, 7.0, 4.0, seed=8)
    assert np.array_equal(a.values, b.values) and np.array_equal(a.row_idx, b.row_idx)
    assert not np.array_equal(a.values, c.values)


def test_water_cutoff_pattern_matches_min_image_distances():
    s = water_system(10, 7.0, 3.5, seed=9)
    pos = s.coords
    d = pos[:, None, :] - pos[None, :, :]
    d -= 7.0 * np.round(d / 7.0)
    dist = np.sqrt((d * d).sum(-1))
    want = dist < 3.5
    got = np.zeros_like(want)
    for j in range(s.nblk):
        got[s.row_idx[s.col_ptr[j]:s.col_ptr[j + 1]], j] = True
    assert np.array_equal(got, want)


def test_random_and_chain_builders():
    s = random_block_system(1, [3, 1, 4], density=1.0, groups="all")
    assert s.ngroups == 1 and s.nnzb == 9
    kd = s.to_dense()
    assert np.array_equal(kd, kd.T)
    c = tb_chain(12, 3, periodic=True, pattern="band")
    assert c.nnzb == 4 * 3
