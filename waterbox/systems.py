"""Builders for block-sparse symmetric test matrices (inputs only).

Every builder returns a :class:`BlockSparse` in BSC form (both triangles
stored).  Randomness comes only from ``numpy.random.default_rng(seed)``
(PCG64) and is drawn in a fixed, documented order so that any consumer
re-creating a system from its seed gets bit-identical arrays.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

# Basis functions per atom (DZVP-like sizes, Sec. V-C mentions DZVP; the
# paper's DBCSR blocks are "typically 5-30 rows and columns", Sec. II-C).
O_BLOCK = 13
H_BLOCK = 5

# Rigid water geometry (angstrom / degrees).
OH_BOND = 0.9572
HOH_ANGLE = 104.52

# Value distributions of the synthetic K.
OFFDIAG_SIGMA = 0.1     # std of off-diagonal block entries before decay
DECAY_LENGTH = 1.5      # K_IJ = exp(-d_IJ / DECAY_LENGTH) * G
DIAG_SIGMA = 0.05       # std of the symmetric noise on diagonal blocks
ONSITE = 0.5            # on-site energies alternate -ONSITE / +ONSITE

# Element-wise decay (opt-in, ``elem_decay=True``): every basis function has a
# range, from compact (core-like) to diffuse, and the off-diagonal element
# (a, b) of block (I, J) decays as exp(-d_IJ / lambda_ab) with lambda_ab the
# mean of the two ranges.  Elements whose magnitude falls to ``eps_filter`` or
# below are set to zero, as the paper's element cutoff does (Sec. V-C, element-
# wise sparsity of the submatrices); the block pattern is unchanged.
O_RANGES = (0.2, 0.2, 0.25, 0.25, 0.25, 0.35, 0.35, 0.35, 0.5, 0.5, 0.5, 0.8, 0.8)
H_RANGES = (0.25, 0.25, 0.35, 0.5, 0.8)


@dataclasses.dataclass
class BlockSparse:
    """A block-sparse symmetric matrix in BSC form plus its submatrix groups."""

    blk_size: np.ndarray          # int32 [nblk]
    col_ptr: np.ndarray           # int64 [nblk + 1]
    row_idx: np.ndarray           # int32 [nnzb], ascending within a column
    values: np.ndarray            # float64, blocks column-major in storage order
    grp_ptr: np.ndarray           # int32 [ngroups + 1]
    grp_blocks: np.ndarray        # int32, block columns of each group
    mu: float = 0.0
    coords: Optional[np.ndarray] = None   # atom positions (angstrom), if any
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nblk(self) -> int:
        return int(self.blk_size.shape[0])

    @property
    def nnzb(self) -> int:
        return int(self.row_idx.shape[0])

    @property
    def n(self) -> int:
        return int(self.blk_size.sum())

    @property
    def ngroups(self) -> int:
        return int(self.grp_ptr.shape[0] - 1)

    def val_off(self) -> np.ndarray:
        """Offset of every stored block in ``values`` (int64 [nnzb + 1])."""
        cols = np.repeat(np.arange(self.nblk), np.diff(self.col_ptr))
        sizes = self.blk_size[self.row_idx].astype(np.int64) * self.blk_size[cols]
        off = np.zeros(self.nnzb + 1, dtype=np.int64)
        np.cumsum(sizes, out=off[1:])
        return off

    def to_dense(self) -> np.ndarray:
        """Dense n x n copy (format conversion only; unstored blocks are 0)."""
        boff = block_offsets(self.blk_size)
        out = np.zeros((self.n, self.n))
        voff = self.val_off()
        for j in range(self.nblk):
            bj = int(self.blk_size[j])
            for p in range(int(self.col_ptr[j]), int(self.col_ptr[j + 1])):
                i = int(self.row_idx[p])
                bi = int(self.blk_size[i])
                blk = self.values[voff[p]:voff[p + 1]].reshape(bj, bi).T
                out[boff[i]:boff[i] + bi, boff[j]:boff[j] + bj] = blk
        return out

    def with_groups(self, groups: Sequence[Sequence[int]]) -> "BlockSparse":
        ptr, blocks = _groups_to_csr(groups)
        return dataclasses.replace(self, grp_ptr=ptr, grp_blocks=blocks)

    def with_values(self, values: np.ndarray) -> "BlockSparse":
        return dataclasses.replace(self, values=np.ascontiguousarray(values, dtype=np.float64))


def block_offsets(blk_size: np.ndarray) -> np.ndarray:
    off = np.zeros(len(blk_size) + 1, dtype=np.int64)
    np.cumsum(np.asarray(blk_size, dtype=np.int64), out=off[1:])
    return off


def _groups_to_csr(groups: Sequence[Sequence[int]]):
    ptr = np.zeros(len(groups) + 1, dtype=np.int32)
    ptr[1:] = np.cumsum([len(g) for g in groups])
    blocks = np.array([b for g in groups for b in g], dtype=np.int32)
    return ptr, blocks


def column_groups(nblk: int):
    """One group per block column (the paper's block-level default, Sec. IV-C)."""
    return _groups_to_csr([[j] for j in range(nblk)])


# ---------------------------------------------------------------------------
# Generic constructor: dense symmetric matrix + block sizes + block mask.
# ---------------------------------------------------------------------------

def dense_to_bsc(kd: np.ndarray, blk_size: Sequence[int], mask: np.ndarray,
                 groups: Optional[Sequence[Sequence[int]]] = None,
                 mu: float = 0.0) -> BlockSparse:
    """Store the blocks of ``kd`` selected by the symmetric ``mask`` in BSC.

    Diagonal blocks are always stored.  ``groups`` defaults to one group per
    block column.
    """
    blk_size = np.asarray(blk_size, dtype=np.int32)
    nblk = len(blk_size)
    mask = np.asarray(mask, dtype=bool).copy()
    if mask.shape != (nblk, nblk) or not np.array_equal(mask, mask.T):
        raise ValueError("mask must be a symmetric nblk x nblk boolean array")
    np.fill_diagonal(mask, True)
    boff = block_offsets(blk_size)
    col_ptr = np.zeros(nblk + 1, dtype=np.int64)
    rows, vals = [], []
    for j in range(nblk):
        ii = np.nonzero(mask[:, j])[0]
        col_ptr[j + 1] = col_ptr[j] + len(ii)
        rows.append(ii.astype(np.int32))
        for i in ii:
            blk = kd[boff[i]:boff[i + 1], boff[j]:boff[j + 1]]
            vals.append(np.asarray(blk, dtype=np.float64).reshape(-1, order="F"))
    if groups is None:
        grp_ptr, grp_blocks = column_groups(nblk)
    else:
        grp_ptr, grp_blocks = _groups_to_csr(groups)
    return BlockSparse(blk_size=blk_size, col_ptr=col_ptr,
                       row_idx=np.concatenate(rows), values=np.concatenate(vals),
                       grp_ptr=grp_ptr, grp_blocks=grp_blocks, mu=mu)


# ---------------------------------------------------------------------------
# 1-D tight-binding chain / ring (closed-form spectra, used as pins).
# ---------------------------------------------------------------------------

def tb_chain(n_sites: int, blk: int, alpha: float = 0.0, beta: float = -1.0,
             periodic: bool = False, pattern: str = "band",
             mu: float = 0.0) -> BlockSparse:
    """H = alpha*I + beta*(shift + shift^T) on ``n_sites`` sites, in blocks of ``blk`` sites.

    ``pattern='band'`` stores the blocks that hold non-zero couplings
    (|I-J| <= 1, plus the wrap-around pair for a ring); ``'dense'`` stores
    every block.  Groups are single block columns.
    """
    if n_sites % blk:
        raise ValueError("n_sites must be a multiple of blk")
    h = alpha * np.eye(n_sites)
    idx = np.arange(n_sites - 1)
    h[idx, idx + 1] = beta
    h[idx + 1, idx] = beta
    if periodic:
        h[0, n_sites - 1] = beta
        h[n_sites - 1, 0] = beta
    nblk = n_sites // blk
    if pattern == "dense":
        mask = np.ones((nblk, nblk), dtype=bool)
    elif pattern == "band":
        ib = np.arange(nblk)
        dist = np.abs(ib[:, None] - ib[None, :])
        if periodic:
            dist = np.minimum(dist, nblk - dist)
        mask = dist <= 1
    else:
        raise ValueError(pattern)
    out = dense_to_bsc(h, [blk] * nblk, mask, mu=mu)
    out.meta = dict(kind="tb_chain", n_sites=n_sites, blk=blk, alpha=alpha,
                    beta=beta, periodic=periodic, pattern=pattern)
    return out


# ---------------------------------------------------------------------------
# Random block-sparse systems with ragged block sizes (parity cases).
# ---------------------------------------------------------------------------

def random_block_system(seed: int, blk_sizes: Sequence[int], density: float = 0.3,
                        coupling: float = 0.05, groups: str | Sequence[Sequence[int]] = "column",
                        mu: float = 0.0) -> BlockSparse:
    """Random symmetric block-sparse K with a gap around ``mu``.

    Draw order from ``default_rng(seed)``: the upper-triangle block mask
    (uniform < density, columns ascending, rows ascending), then the dense
    n x n Gaussian coupling matrix, then the diagonal signs.  The diagonal
    holds +-ONSITE (random signs) + mu, couplings are N(0, coupling^2) and
    symmetrised, so the spectrum of every principal submatrix avoids mu by
    roughly ONSITE minus the coupling norm.
    """
    rng = np.random.default_rng(seed)
    blk_sizes = np.asarray(blk_sizes, dtype=np.int32)
    nblk = len(blk_sizes)
    up = rng.uniform(size=(nblk, nblk)) < density
    mask = np.triu(up, 1)
    mask = mask | mask.T
    n = int(blk_sizes.sum())
    g = rng.normal(0.0, coupling, size=(n, n))
    g = (g + g.T) * 0.5
    signs = np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    kd = g + np.diag(signs * ONSITE + mu)
    if isinstance(groups, str):
        if groups == "column":
            grp = [[j] for j in range(nblk)]
        elif groups == "pairs":
            grp = [list(range(j, min(j + 2, nblk))) for j in range(0, nblk, 2)]
        elif groups == "all":
            grp = [list(range(nblk))]
        else:
            raise ValueError(groups)
    else:
        grp = [list(x) for x in groups]
    out = dense_to_bsc(kd, blk_sizes, mask, groups=grp, mu=mu)
    out.meta = dict(kind="random_block", seed=seed, density=density, coupling=coupling)
    return out


# ---------------------------------------------------------------------------
# Water-like systems.
# ---------------------------------------------------------------------------

# name -> (molecules, box length in angstrom, cutoff in angstrom, seed)
WATER_CONFIGS = {
    # 16 molecules, 368 basis functions, 4 A cutoff (> L/2: minimum image only)
    "water16": dict(n_mol=16, box=7.8, r_cut=4.0, seed=1),
    # 1024 molecules, 23552 basis functions, liquid density
    "water1024": dict(n_mol=1024, box=31.3, r_cut=6.0, seed=2),
    # 256 molecules, 5888 basis functions, box chosen for liquid density
    "water256": dict(n_mol=256, box=19.7, r_cut=6.0, seed=4),
    # 6912 molecules, 158976 basis functions
    "water6912": dict(n_mol=6912, box=59.6, r_cut=7.0, seed=5),
    # element-sparse variants: same geometry, per-function ranges, element cutoff 1e-5
    "water16e": dict(n_mol=16, box=7.8, r_cut=4.0, seed=1, elem_decay=True, eps_filter=1e-5),
    "water256e": dict(n_mol=256, box=19.7, r_cut=6.0, seed=4, elem_decay=True, eps_filter=1e-5),
    "water1024e": dict(n_mol=1024, box=31.3, r_cut=6.0, seed=2, elem_decay=True, eps_filter=1e-5),
}


def water_config(name: str, **over) -> BlockSparse:
    kw = dict(WATER_CONFIGS[name])
    kw.update(over)
    sysm = water_system(**kw)
    sysm.meta["config"] = name
    return sysm


def _quat_to_rot(q: np.ndarray) -> np.ndarray:
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    r = np.empty((q.shape[0], 3, 3))
    r[:, 0, 0] = 1 - 2 * (y * y + z * z)
    r[:, 0, 1] = 2 * (x * y - z * w)
    r[:, 0, 2] = 2 * (x * z + y * w)
    r[:, 1, 0] = 2 * (x * y + z * w)
    r[:, 1, 1] = 1 - 2 * (x * x + z * z)
    r[:, 1, 2] = 2 * (y * z - x * w)
    r[:, 2, 0] = 2 * (x * z - y * w)
    r[:, 2, 1] = 2 * (y * z + x * w)
    r[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def _min_image_pairs(pos: np.ndarray, box: float, r_cut: float):
    """All pairs i < j with minimum-image distance < r_cut, sorted by (j, i).

    A periodic k-d tree proposes the candidate pairs (with a slightly larger
    radius); the distance that decides is then computed for each candidate as
    d = |pos_i - pos_j - box * round((pos_i - pos_j) / box)|.
    """
    from scipy.spatial import cKDTree
    wrapped = np.where(pos >= box, pos - box, pos)        # mod() may round up to box
    tree = cKDTree(wrapped, boxsize=box)
    cand = tree.query_pairs(r_cut * (1.0 + 1e-9), output_type="ndarray")
    i = cand[:, 0].astype(np.int64)
    j = cand[:, 1].astype(np.int64)
    delta = pos[i] - pos[j]
    delta -= box * np.round(delta / box)
    d = np.sqrt((delta * delta).sum(-1))
    keep = d < r_cut
    i, j, d = i[keep], j[keep], d[keep]
    order = np.lexsort((i, j))
    return i[order].astype(np.int64), j[order].astype(np.int64), d[order]


def water_system(n_mol: int, box: float, r_cut: float, seed: int,
                 pattern: str = "cutoff", elem_decay: bool = False,
                 eps_filter: float = 0.0) -> BlockSparse:
    """Seeded water-like block-sparse K (one block per atom, groups = molecules).

    Recipe (all draws from ``default_rng(seed)``, in this order):

    1. Oxygen sites: n_side = smallest integer with n_side^3 >= n_mol,
       a = box / n_side; ``permutation(n_side^3)[:n_mol]`` picks the
       simple-cubic sites, kept in ascending (lexicographic) site order so
       that neighbouring molecules get neighbouring indices (Sec. IV-B).
    2. Jitter: ``uniform(-0.15a, 0.15a, (n_mol, 3))`` added to the site
       centres (site + 0.5) * a.
    3. Orientation: ``normal(size=(n_mol, 4))`` normalised to a unit
       quaternion rotates the rigid O-H-H geometry; positions wrap into the box.
    4. Pattern: block (I, J) is stored iff the minimum-image distance
       d_IJ < r_cut (``pattern='cutoff'``); ``'blockdiag'`` stores only
       intramolecular blocks; ``'dense'`` stores every block.
    5. Off-diagonal values: one ``normal(0, 0.1, total)`` call covers all
       stored upper blocks (I < J) in storage order (columns ascending, rows
       ascending), each block column-major; K_IJ = exp(-d_IJ/1.5) * G and
       K_JI = K_IJ^T.  With ``elem_decay`` the factor is exp(-d_IJ/lambda_ab)
       per element instead (lambda_ab the mean of the two basis functions'
       ranges, O_RANGES / H_RANGES); the draws are the same.
    6. Diagonal blocks: one ``normal(0, 0.05, total)`` call gives the upper
       triangle (diagonal included, column by column) of a symmetric noise
       block for every atom in order; on-site energies are -0.5 Ha for even
       global basis index and +0.5 Ha for odd ones, so exactly n/2 of each.
    7. Element cutoff: every stored value with magnitude <= eps_filter is
       set to zero (eps_filter = 0: none).
    """
    rng = np.random.default_rng(seed)
    n_side = 1
    while n_side ** 3 < n_mol:
        n_side += 1
    a = box / n_side
    sites = np.sort(rng.permutation(n_side ** 3)[:n_mol])
    ix, rem = np.divmod(sites, n_side * n_side)
    iy, iz = np.divmod(rem, n_side)
    centre = (np.stack([ix, iy, iz], axis=1) + 0.5) * a
    centre = centre + rng.uniform(-0.15 * a, 0.15 * a, size=(n_mol, 3))
    rot = _quat_to_rot(rng.normal(size=(n_mol, 4)))
    half = math.radians(HOH_ANGLE) / 2.0
    local = np.array([[0.0, 0.0, 0.0],
                      [OH_BOND * math.sin(half), 0.0, OH_BOND * math.cos(half)],
                      [-OH_BOND * math.sin(half), 0.0, OH_BOND * math.cos(half)]])
    pos = centre[:, None, :] + np.einsum("mij,aj->mai", rot, local)
    pos = np.mod(pos.reshape(-1, 3), box)
    natom = 3 * n_mol
    blk_size = np.tile(np.array([O_BLOCK, H_BLOCK, H_BLOCK], dtype=np.int32), n_mol)
    mol = np.repeat(np.arange(n_mol), 3)

    if pattern == "cutoff":
        pi, pj, pd = _min_image_pairs(pos, box, r_cut)
    elif pattern in ("blockdiag", "dense"):
        ai, aj = np.triu_indices(natom, 1)
        if pattern == "blockdiag":
            keep = mol[ai] == mol[aj]
            ai, aj = ai[keep], aj[keep]
        delta = pos[ai] - pos[aj]
        delta -= box * np.round(delta / box)
        pd = np.sqrt((delta * delta).sum(-1))
        order = np.lexsort((ai, aj))
        pi, pj, pd = ai[order].astype(np.int64), aj[order].astype(np.int64), pd[order]
    else:
        raise ValueError(pattern)

    # Upper off-diagonal blocks, storage order (j ascending, i ascending).
    bi = blk_size[pi].astype(np.int64)
    bj = blk_size[pj].astype(np.int64)
    up_sz = bi * bj
    up_off = np.zeros(len(pi) + 1, dtype=np.int64)
    np.cumsum(up_sz, out=up_off[1:])
    g_off = rng.normal(0.0, OFFDIAG_SIGMA, size=int(up_off[-1]))
    if elem_decay:
        ranges = {O_BLOCK: np.array(O_RANGES), H_BLOCK: np.array(H_RANGES)}
        for (bsi, bsj) in {(int(x), int(y)) for x, y in zip(bi, bj)}:
            sel = np.nonzero((bi == bsi) & (bj == bsj))[0]
            # lambda of element (a, b) of a bsi x bsj block, column-major
            lam = (0.5 * (ranges[bsi][:, None] + ranges[bsj][None, :])).reshape(-1, order="F")
            idx = up_off[sel][:, None] + np.arange(bsi * bsj)[None, :]
            g_off[idx] *= np.exp(-pd[sel][:, None] / lam[None, :])
    else:
        scale = np.repeat(np.exp(-pd / DECAY_LENGTH), up_sz)
        g_off *= scale

    # Diagonal noise, upper triangle incl. diagonal, column by column.
    tri = blk_size.astype(np.int64) * (blk_size + 1) // 2
    tri_off = np.zeros(natom + 1, dtype=np.int64)
    np.cumsum(tri, out=tri_off[1:])
    g_diag = rng.normal(0.0, DIAG_SIGMA, size=int(tri_off[-1]))

    # Full pattern: both triangles + diagonal, sorted by (col, row).
    all_i = np.concatenate([pi, pj, np.arange(natom)])
    all_j = np.concatenate([pj, pi, np.arange(natom)])
    kind = np.concatenate([np.zeros(len(pi), np.int8), np.ones(len(pi), np.int8),
                           np.full(natom, 2, np.int8)])
    src = np.concatenate([np.arange(len(pi)), np.arange(len(pi)), np.arange(natom)])
    order = np.lexsort((all_i, all_j))
    all_i, all_j, kind, src = all_i[order], all_j[order], kind[order], src[order]
    col_ptr = np.zeros(natom + 1, dtype=np.int64)
    np.cumsum(np.bincount(all_j, minlength=natom), out=col_ptr[1:])
    sz = blk_size[all_i].astype(np.int64) * blk_size[all_j]
    voff = np.zeros(len(all_i) + 1, dtype=np.int64)
    np.cumsum(sz, out=voff[1:])
    values = np.empty(int(voff[-1]))
    boff = block_offsets(blk_size)

    for (bsi, bsj) in {(int(x), int(y)) for x in np.unique(blk_size) for y in np.unique(blk_size)}:
        sel = (blk_size[all_i] == bsi) & (blk_size[all_j] == bsj)
        r = np.arange(bsi)[:, None]
        c = np.arange(bsj)[None, :]
        local_cm = (r + c * bsi).reshape(-1)          # destination, column-major bsi x bsj
        # upper blocks: source is the drawn block, column-major bsi x bsj
        s_up = sel & (kind == 0)
        if s_up.any():
            dst = voff[:-1][s_up][:, None] + local_cm[None, :]
            srci = up_off[src[s_up]][:, None] + local_cm[None, :]
            values[dst] = g_off[srci]
        # lower blocks: K_IJ = (K_JI)^T, K_JI drawn column-major bsj x bsi
        s_lo = sel & (kind == 1)
        if s_lo.any():
            dst = voff[:-1][s_lo][:, None] + local_cm[None, :]
            tr = (c + r * bsj).reshape(-1)
            srci = up_off[src[s_lo]][:, None] + tr[None, :]
            values[dst] = g_off[srci]
        # diagonal blocks
        s_d = sel & (kind == 2)
        if s_d.any() and bsi == bsj:
            rr = np.minimum(r, c)
            cc = np.maximum(r, c)
            tri_idx = (cc * (cc + 1) // 2 + rr).reshape(-1)
            atoms = src[s_d]
            dst = voff[:-1][s_d][:, None] + local_cm[None, :]
            vals = g_diag[tri_off[atoms][:, None] + tri_idx[None, :]]
            gidx = boff[atoms][:, None] + np.arange(bsi)[None, :]
            onsite = np.where(gidx % 2 == 0, -ONSITE, ONSITE)
            on_diag = (r == c).reshape(-1)
            vals[:, on_diag] += onsite
            values[dst] = vals

    if eps_filter > 0.0:
        values[np.abs(values) <= eps_filter] = 0.0

    grp_ptr = np.arange(0, natom + 1, 3, dtype=np.int32)
    grp_blocks = np.arange(natom, dtype=np.int32)
    out = BlockSparse(blk_size=blk_size, col_ptr=col_ptr, row_idx=all_i.astype(np.int32),
                      values=values, grp_ptr=grp_ptr, grp_blocks=grp_blocks, mu=0.0,
                      coords=pos)
    out.meta = dict(kind="water", n_mol=n_mol, box=box, r_cut=r_cut, seed=seed,
                    pattern=pattern, elem_decay=elem_decay, eps_filter=eps_filter)
    return out
