"""Host: splitting submatrices into sub-submatrices (Sec. IV-C, "Splitting up
submatrices") -- the oracle's split method against what the paper and the
mathematics fix, and the library's construction of the split problem against
a direct numpy construction.

Oracle pins: with eps = 0 on blocks without zero elements every sub-submatrix
is its block column's submatrix (so D equals the block-column submatrix
method); on a chain stored in dense blocks every sub-submatrix is a 2- or
3-site chain with a closed-form density; with eps above every off-diagonal
magnitude D is the diagonal step function; the result does not depend on how
block columns are grouped; and it equals the plain submatrix method applied to
the element-level matrix with single-column groups.
"""

import math

import numpy as np
import pytest

from waterbox import water_config, random_block_system, tb_chain, dense_to_bsc
from waterbox.systems import block_offsets


@pytest.fixture(scope="module")
def smx():
    import paper_2004_10811_amd as smx
    smx.load_library()
    return smx


def dense_d(s, d_values):
    boff = block_offsets(s.blk_size)
    voff = s.val_off()
    out = np.full((s.n, s.n), np.nan)
    for j in range(s.nblk):
        for p in range(int(s.col_ptr[j]), int(s.col_ptr[j + 1])):
            i = int(s.row_idx[p])
            out[boff[i]:boff[i + 1], boff[j]:boff[j + 1]] = d_values[voff[p]:voff[p + 1]].reshape(
                s.blk_size[i], s.blk_size[j], order="F")
    return out


def test_eps_zero_equals_block_column_submatrices(oracle_lib):
    s = random_block_system(3, [7, 3, 11, 5, 9, 2, 6], density=0.5, groups="column", mu=0.02)
    a = oracle_lib.split_submatrix(s, 0.0)
    b = oracle_lib.submatrix(s)
    assert np.abs(a.d_values - b.d_values).max() <= 1e-13
    assert abs(a.n_elec - b.n_elec) <= 1e-12 and abs(a.energy - b.energy) <= 1e-12


def test_chain_in_dense_blocks_closed_form(oracle_lib):
    """Open chain alpha = 0.3, beta = -1, 12 sites in 4-site blocks, every block
    stored: the sub-submatrix of an interior site is the 3-site chain, whose only
    occupied state (alpha + sqrt2 beta < 0) is (1, sqrt2, 1) / 2, so D's column is
    (sqrt2/4, 1/2, sqrt2/4); an end site gets the 2-site chain, column (1/2, 1/2)."""
    s = tb_chain(12, 4, 0.3, -1.0, periodic=False, pattern="dense")
    r = oracle_lib.split_submatrix(s, 0.0)
    d = dense_d(s, r.d_values)
    ref = np.zeros((12, 12))
    for c in range(12):
        if c in (0, 11):
            nb = 1 if c == 0 else 10
            ref[c, c] = ref[nb, c] = 0.5
        else:
            ref[c, c] = 0.5
            ref[c - 1, c] = ref[c + 1, c] = math.sqrt(2) / 4
    assert np.abs(d - ref).max() <= 1e-14
    assert abs(r.n_elec - 6.0) <= 1e-13
    e_ref = sum(ref[r_, c] * s.to_dense()[r_, c] for r_ in range(12) for c in range(12))
    assert abs(r.energy - e_ref) <= 1e-13


def test_large_eps_gives_the_diagonal_step(oracle_lib):
    s = random_block_system(4, [5, 8, 3, 6], density=0.6, groups="pairs", mu=0.05)
    kd = s.to_dense()
    r = oracle_lib.split_submatrix(s, 1e9)
    d = dense_d(s, r.d_values)
    diag = np.where(np.diag(kd) - 0.05 < 0, 1.0, 0.0)
    assert np.array_equal(np.diag(d), diag)
    off = d - np.diag(np.diag(d))
    assert np.nanmax(np.abs(off)) == 0.0
    assert r.n_elec == diag.sum()


def test_independent_of_grouping(oracle_lib):
    s = water_config("water16e")
    eps = 1e-5
    mol = oracle_lib.split_submatrix(s, eps, which=[0, 5])
    single = s.with_groups([[j] for j in range(s.nblk)])
    cols = oracle_lib.split_submatrix(single, eps, which=[0, 1, 2, 15, 16, 17])
    ok = ~np.isnan(mol.d_values)
    assert np.array_equal(ok, ~np.isnan(cols.d_values))
    assert np.abs(mol.d_values[ok] - cols.d_values[ok]).max() <= 1e-13


def element_level(s, eps):
    """The element-level matrix of the split (numpy): 1 x 1 blocks, column c keeps
    r = c and the rows of its stored blocks with |K_rc| > eps."""
    kd = s.to_dense()
    boff = block_offsets(s.blk_size)
    stored = np.zeros((s.n, s.n), dtype=bool)
    for j in range(s.nblk):
        for p in range(int(s.col_ptr[j]), int(s.col_ptr[j + 1])):
            i = int(s.row_idx[p])
            stored[boff[i]:boff[i + 1], boff[j]:boff[j + 1]] = True
    keep = stored & (np.abs(kd) > eps)
    np.fill_diagonal(keep, True)
    return kd, keep


def test_split_equals_element_level_submatrix(oracle_lib):
    s = water_config("water16e")
    eps = 1e-5
    kd, keep = element_level(s, eps)
    e = dense_to_bsc(kd, [1] * s.n, keep, mu=s.mu)
    pick = [3, 40, 41, 200, 367]
    a = oracle_lib.submatrix(e, which=pick)
    b = oracle_lib.split_submatrix(s, eps)
    db = dense_d(s, b.d_values)
    da = dense_d(e, a.d_values)
    for c in pick:
        rows = np.nonzero(keep[:, c])[0]
        assert np.abs(da[rows, c] - db[rows, c]).max() <= 1e-13
        dropped = np.nonzero(~keep[:, c] & ~np.isnan(db[:, c]))[0]
        assert np.all(db[dropped, c] == 0.0)


@pytest.mark.parametrize("case", ["water16e", "ragged"])
def test_library_split_problem(smx, case):
    if case == "ragged":
        s = random_block_system(9, [13, 5, 5, 17, 9, 31, 22], density=0.5, groups="pairs")
        s = s.with_values(np.where(np.abs(s.values) < 0.02, 0.0, s.values))
        eps = 0.03
    else:
        s = water_config(case)
        eps = 1e-5
    kd, keep = element_level(s, eps)
    sp = smx.split_columns(s, eps, merge=False)
    assert np.array_equal(sp.col_ptr, np.concatenate([[0], np.cumsum(keep.sum(0))]))
    for c in range(s.n):
        rows = sp.row_idx[sp.col_ptr[c]:sp.col_ptr[c + 1]]
        assert np.array_equal(rows, np.nonzero(keep[:, c])[0])
        assert np.array_equal(sp.values[sp.col_ptr[c]:sp.col_ptr[c + 1]], kd[rows, c])
    assert np.array_equal(s.values[sp.src], sp.values)
    assert len(np.unique(sp.src)) == len(sp.src)
    assert np.array_equal(sp.grp_ptr, np.arange(s.n + 1)) and np.array_equal(sp.grp_blocks, np.arange(s.n))
    m = smx.split_columns(s, eps, merge=True)
    assert np.array_equal(m.row_idx, sp.row_idx) and np.array_equal(m.src, sp.src)
    for g in range(len(m.grp_ptr) - 1):
        cols = m.grp_blocks[m.grp_ptr[g]:m.grp_ptr[g + 1]]
        first = sp.row_idx[sp.col_ptr[cols[0]]:sp.col_ptr[cols[0] + 1]]
        for c in cols[1:]:
            assert np.array_equal(sp.row_idx[sp.col_ptr[c]:sp.col_ptr[c + 1]], first)
    print(f"{case}: {s.n} columns, {len(sp.values)} of {len(s.values)} values kept, "
          f"{len(m.grp_ptr) - 1} merged groups")


def test_split_rejects_bad_input(smx):
    s = water_config("water16")
    with pytest.raises(smx.SmxError) as ei:
        smx.split_columns(s, -1.0)
    assert ei.value.code == smx.SMX_E_INVALID
    bad = s.with_values(s.values)
    bad.row_idx = s.row_idx.copy()
    bad.row_idx[1], bad.row_idx[2] = bad.row_idx[2], bad.row_idx[1]
    with pytest.raises(smx.SmxError):
        smx.split_columns(bad, 0.0)
