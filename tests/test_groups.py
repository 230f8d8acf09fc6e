"""Host: group selection (Sec. IV-C) -- the estimated speedup of combining block
columns into submatrices (Eq. estimatedspeedup) and the k-means proposal of
such combinations from the block columns' positions.

Pins: S = 1 when every group is one block column; S of one group holding the
whole matrix is sum_j n_j^3 / n^3; S of any grouping equals a direct numpy
evaluation of the definition (union of the stored block rows of the group's
columns); k-means recovers well-separated blobs (also one wrapped across a
periodic box) with the partition scikit-learn's Lloyd iteration finds; its
result is a fixed point of Lloyd's map; it is deterministic for a seed, a valid
partition, and refuses bad arguments.
"""

import numpy as np
import pytest

from waterbox import water_config, random_block_system


@pytest.fixture(scope="module")
def smx():
    import paper_2004_10811_amd as smx
    smx.load_library()
    return smx


def dims_numpy(s, groups):
    out = []
    for cols in groups:
        rows = set()
        for j in cols:
            rows.update(int(i) for i in s.row_idx[s.col_ptr[j]:s.col_ptr[j + 1]])
        out.append(int(s.blk_size[sorted(rows)].sum()))
    return np.array(out, dtype=np.float64)


def csr(groups):
    gp = np.zeros(len(groups) + 1, np.int32)
    gp[1:] = np.cumsum([len(g) for g in groups])
    return gp, np.concatenate([np.asarray(g, np.int32) for g in groups])


def groups_of(gp, gb):
    return [list(gb[gp[g]:gp[g + 1]]) for g in range(len(gp) - 1)]


def test_single_columns_give_one(smx):
    s = water_config("water16")
    gp, gb = csr([[j] for j in range(s.nblk)])
    sp, work = smx.group_speedup(s, gp, gb)
    assert sp == 1.0
    assert work == float((dims_numpy(s, [[j] for j in range(s.nblk)]) ** 3).sum())


def test_whole_matrix_closed_form(smx):
    s = random_block_system(5, [7, 3, 11, 5, 9, 2], density=0.4, groups="column")
    gp, gb = csr([list(range(s.nblk))])
    sp, work = smx.group_speedup(s, gp, gb)
    nj = dims_numpy(s, [[j] for j in range(s.nblk)])
    assert work == float(s.n) ** 3
    assert sp == pytest.approx((nj ** 3).sum() / float(s.n) ** 3, rel=1e-15)


@pytest.mark.parametrize("case", ["water16", "water256", "ragged"])
def test_speedup_matches_definition(smx, case):
    if case == "ragged":
        s = random_block_system(7, [13, 5, 5, 17, 9, 31, 22, 13, 27, 11, 5, 25] * 2, density=0.35, groups="pairs")
    else:
        s = water_config(case)
    groups = groups_of(s.grp_ptr, s.grp_blocks)
    sp, work = smx.group_speedup(s)
    ng = dims_numpy(s, groups)
    nj = dims_numpy(s, [[j] for j in range(s.nblk)])
    assert work == pytest.approx(float((ng ** 3).sum()), rel=1e-15)
    assert sp == pytest.approx(float((nj ** 3).sum() / (ng ** 3).sum()), rel=1e-14)
    # invariant under the order of groups and of columns inside a group
    rng = np.random.default_rng(3)
    shuffled = [list(rng.permutation(g)) for g in groups]
    rng.shuffle(shuffled)
    assert smx.group_speedup(s, *csr(shuffled))[0] == pytest.approx(sp, rel=1e-14)


def test_speedup_rejects_bad_groups(smx):
    s = water_config("water16")
    for groups in ([list(range(s.nblk - 1))], [[0, 0]] + [[j] for j in range(1, s.nblk)]):
        with pytest.raises(smx.SmxError) as ei:
            smx.group_speedup(s, *csr(groups))
        assert ei.value.code == smx.SMX_E_INVALID


def blobs(rng, k, per, spread, box=None, sep=12.0):
    # centres drawn one by one, redrawn while closer than sep to an earlier one
    # (minimum image in a box) or to the box corner
    ext = 100.0 if box is None else box
    centres = []
    while len(centres) < k:
        c = rng.uniform(0.0, ext, size=3)
        others = centres + ([np.zeros(3)] if box is not None else [])
        d = np.array([c - o for o in others]) if others else np.zeros((0, 3))
        if box is not None:
            d -= box * np.round(d / box)
        if not len(d) or np.sqrt((d * d).sum(1)).min() >= sep:
            centres.append(c)
    centres = np.array(centres)
    pts = (centres[:, None, :] + rng.normal(0.0, spread, size=(k, per, 3))).reshape(-1, 3)
    label = np.repeat(np.arange(k), per)
    perm = rng.permutation(len(pts))
    pts, label = pts[perm], label[perm]
    if box is not None:
        pts = np.mod(pts, box)
    return pts, label, centres


def same_partition(gp, gb, label):
    # every group carries one label and every label one group
    seen = {}
    for g, cols in enumerate(groups_of(gp, gb)):
        labs = set(int(label[c]) for c in cols)
        if len(labs) != 1:
            return False
        lab = labs.pop()
        if lab in seen:
            return False
        seen[lab] = g
    return len(seen) == len(set(label.tolist()))


def valid_partition(gp, gb, nb):
    assert gp[0] == 0 and gp[-1] == nb and np.all(np.diff(gp) > 0)
    assert sorted(gb.tolist()) == list(range(nb))
    for cols in groups_of(gp, gb):
        assert list(cols) == sorted(cols)
    firsts = [cols[0] for cols in groups_of(gp, gb)]
    assert firsts == sorted(firsts)


def test_kmeans_recovers_blobs_like_sklearn(smx):
    from sklearn.cluster import KMeans
    rng = np.random.default_rng(11)
    pts, label, _ = blobs(rng, 12, 25, 1.0)
    gp, gb = smx.group_kmeans(pts, 12, seed=5)
    valid_partition(gp, gb, len(pts))
    assert same_partition(gp, gb, label)
    sk = KMeans(n_clusters=12, n_init=10, random_state=0).fit(pts)
    assert same_partition(gp, gb, sk.labels_)


def test_kmeans_periodic_wraps(smx):
    """A blob centred on a corner of the box is split into eight pieces by the
    wrap; the minimum-image metric and circular means keep it one cluster."""
    rng = np.random.default_rng(12)
    box = 40.0
    pts, label, _ = blobs(rng, 5, 30, 0.8, box=box)
    corner = np.mod(rng.normal(0.0, 0.8, size=(30, 3)), box)
    pts = np.vstack([pts, corner])
    label = np.concatenate([label, np.full(30, 5)])
    assert (corner > box / 2).any() and (corner < box / 2).any()
    gp, gb = smx.group_kmeans(pts, 6, box=box, seed=1)
    valid_partition(gp, gb, len(pts))
    assert same_partition(gp, gb, label)
    # without the box the corner blob is torn apart
    gp0, gb0 = smx.group_kmeans(pts, 6, seed=1)
    assert not same_partition(gp0, gb0, label)


def lloyd_fixed_point(pts, gp, gb, box):
    groups = groups_of(gp, gb)
    cen = []
    for cols in groups:
        p = pts[cols]
        if box > 0:
            w = 2 * np.pi / box
            a = np.arctan2(np.sin(w * p).sum(0), np.cos(w * p).sum(0)) / w
            cen.append(np.mod(a, box))
        else:
            cen.append(p.mean(0))
    cen = np.array(cen)
    d = pts[:, None, :] - cen[None, :, :]
    if box > 0:
        d -= box * np.round(d / box)
    d2 = (d * d).sum(-1)
    own = np.empty(len(pts), int)
    for g, cols in enumerate(groups):
        own[cols] = g
    return np.all(d2[np.arange(len(pts)), own] <= d2.min(1) * (1 + 1e-12) + 1e-12)


@pytest.mark.parametrize("box", [0.0, 19.7])
def test_kmeans_water_is_a_lloyd_fixed_point(smx, box):
    s = water_config("water256")
    gp, gb = smx.group_kmeans(s.coords, 128, box=box, seed=2, max_iter=500)
    valid_partition(gp, gb, s.nblk)
    assert lloyd_fixed_point(s.coords, gp, gb, box)
    again = smx.group_kmeans(s.coords, 128, box=box, seed=2, max_iter=500)
    assert np.array_equal(gp, again[0]) and np.array_equal(gb, again[1])
    sp, _ = smx.group_speedup(s, gp, gb)
    print(f"water256 k-means 128 (box {box}): {len(gp) - 1} groups, S = {sp:.3f}, "
          f"molecules S = {smx.group_speedup(s)[0]:.3f}")
    assert sp > 1.0


def test_kmeans_edge_cases(smx):
    pts = np.array([[0.0, 0.0, 0.0]] * 4 + [[5.0, 0.0, 0.0]] * 3)
    gp, gb = smx.group_kmeans(pts, 1)
    assert gp.tolist() == [0, 7] and gb.tolist() == list(range(7))
    gp, gb = smx.group_kmeans(pts, 7)              # duplicates: at most 2 distinct clusters are non-empty
    valid_partition(gp, gb, 7)
    assert len(gp) - 1 == 2 and same_partition(gp, gb, np.array([0] * 4 + [1] * 3))
    gp, gb = smx.group_kmeans(pts[:1], 1)
    assert gp.tolist() == [0, 1] and gb.tolist() == [0]
    for args in (dict(coords=pts, nclusters=0), dict(coords=pts, nclusters=8),
                 dict(coords=pts, nclusters=2, box=-1.0), dict(coords=pts, nclusters=2, max_iter=0)):
        with pytest.raises(smx.SmxError) as ei:
            smx.group_kmeans(**args)
        assert ei.value.code == smx.SMX_E_INVALID
    bad = pts.copy()
    bad[3, 1] = np.nan
    with pytest.raises(smx.SmxError) as ei:
        smx.group_kmeans(bad, 2)
    assert ei.value.code == smx.SMX_E_NONFINITE
