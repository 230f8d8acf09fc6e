"""TEST INFRASTRUCTURE ONLY: ctypes wrapper of the plain C FP64 oracle.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
this package never imports the product library.

The oracle evaluates the submatrix method with the sign function taken from
a cyclic Jacobi eigendecomposition (see ``smx_oracle.c`` for the passages of
the paper each step follows).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "smx_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP over groups)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class GroupInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nrow_blk", ctypes.c_int32),
                ("sweeps", ctypes.c_int32), ("n_neg", ctypes.c_int32),
                ("n_zero", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("min_abs_lambda", ctypes.c_double), ("max_abs_lambda", ctypes.c_double),
                ("inf_norm", ctypes.c_double), ("eig_residual", ctypes.c_double),
                ("orth_residual", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.oracle_jacobi.argtypes = [i32, P(f64), P(f64), P(f64), i32]
        L.oracle_jacobi.restype = i32
        L.oracle_dense_map.argtypes = [i32, P(f64), i32, f64, P(f64), P(f64), P(f64)]
        L.oracle_dense_map.restype = i32
        L.oracle_group_dims.argtypes = [i32, P(i32), P(i64), P(i32), i32, P(i32), P(i32), P(i32), P(i32)]
        L.oracle_group_dims.restype = i32
        L.oracle_submatrix.argtypes = [i32, P(i32), P(i64), P(i32), P(f64), i32, P(i32), P(i32),
                                       f64, f64, P(i32), i32, i32, P(f64), P(f64), P(f64),
                                       P(GroupInfo)]
        L.oracle_submatrix.restype = i32
        L.oracle_group_eig.argtypes = [i32, P(i32), P(i64), P(i32), P(f64), i32, P(i32), f64,
                                       P(i32), P(f64), P(f64), P(GroupInfo)]
        L.oracle_group_eig.restype = i32
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def jacobi(a: np.ndarray, max_sweeps: int = 60):
    """Eigenpairs of a symmetric matrix: (lam ascending, Q, sweeps)."""
    a = np.asfortranarray(a, dtype=np.float64).copy(order="F")
    n = a.shape[0]
    lam = np.zeros(n)
    q = np.zeros((n, n), order="F")
    sw = lib().oracle_jacobi(n, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             _p(lam, ctypes.c_double),
                             q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), max_sweeps)
    return lam, q, int(sw)


def _dense_map(a, mode, kT):
    a = np.asfortranarray(a, dtype=np.float64)
    n = a.shape[0]
    out = np.zeros((n, n), order="F")
    st = lib().oracle_dense_map(n, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), mode, kT,
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, None)
    if st != 0:
        raise RuntimeError(f"oracle_dense_map failed: {st}")
    return np.array(out)


def dense_sign(a: np.ndarray) -> np.ndarray:
    """sign(A) of a symmetric matrix with the zero-eigenvalue extension."""
    return _dense_map(a, 0, 0.0)


def dense_density(a: np.ndarray, kT: float = 0.0) -> np.ndarray:
    """D = Q occ(Lambda) Q^T of a symmetric (already shifted) matrix."""
    return _dense_map(a, 1, kT)


def _bsc_args(s):
    blk = np.ascontiguousarray(s.blk_size, dtype=np.int32)
    cp = np.ascontiguousarray(s.col_ptr, dtype=np.int64)
    ri = np.ascontiguousarray(s.row_idx, dtype=np.int32)
    gp = np.ascontiguousarray(s.grp_ptr, dtype=np.int32)
    gb = np.ascontiguousarray(s.grp_blocks, dtype=np.int32)
    return blk, cp, ri, gp, gb


def group_dims(s):
    """(n_g, |R(g)|) for every group of a BlockSparse system."""
    blk, cp, ri, gp, gb = _bsc_args(s)
    ng = s.ngroups
    n_out = np.zeros(ng, dtype=np.int32)
    m_out = np.zeros(ng, dtype=np.int32)
    st = lib().oracle_group_dims(s.nblk, _p(blk, ctypes.c_int32), _p(cp, ctypes.c_int64),
                                 _p(ri, ctypes.c_int32), ng, _p(gp, ctypes.c_int32),
                                 _p(gb, ctypes.c_int32), _p(n_out, ctypes.c_int32),
                                 _p(m_out, ctypes.c_int32))
    if st != 0:
        raise RuntimeError(f"oracle_group_dims failed: {st}")
    return n_out, m_out


@dataclass
class OracleResult:
    d_values: np.ndarray      # K's layout; NaN outside the processed groups' columns
    n_elec: float             # Tr D over the processed columns
    energy: float             # Tr(DK) over the processed columns
    info: list                # per processed group: dict of GroupInfo fields
    groups: np.ndarray        # processed group ids


def submatrix(s, mu: float | None = None, kT: float = 0.0, which=None,
              nthreads: int | None = None, values: np.ndarray | None = None) -> OracleResult:
    """Run the submatrix method (Jacobi sign) on a BlockSparse system."""
    blk, cp, ri, gp, gb = _bsc_args(s)
    vals = _f64(s.values if values is None else values)
    mu = s.mu if mu is None else mu
    if which is None:
        which_arr = np.arange(s.ngroups, dtype=np.int32)
        wptr = None
    else:
        which_arr = np.ascontiguousarray(which, dtype=np.int32)
        wptr = _p(which_arr, ctypes.c_int32)
    nj = len(which_arr)
    d = np.full(vals.shape, np.nan)
    info = (GroupInfo * max(nj, 1))()
    n_e = ctypes.c_double()
    e_e = ctypes.c_double()
    nth = nthreads if nthreads else (os.cpu_count() or 1)
    st = lib().oracle_submatrix(s.nblk, _p(blk, ctypes.c_int32), _p(cp, ctypes.c_int64),
                                _p(ri, ctypes.c_int32), _p(vals, ctypes.c_double), s.ngroups,
                                _p(gp, ctypes.c_int32), _p(gb, ctypes.c_int32), float(mu),
                                float(kT), wptr, nj, int(nth), _p(d, ctypes.c_double),
                                ctypes.byref(n_e), ctypes.byref(e_e), info)
    if st != 0:
        raise RuntimeError(f"oracle_submatrix failed: {st}")
    recs = [{f: getattr(info[i], f) for f, _ in GroupInfo._fields_} for i in range(nj)]
    return OracleResult(d, n_e.value, e_e.value, recs, which_arr)


def group_eig(s, g: int, mu: float | None = None, values: np.ndarray | None = None):
    """(R(g), lam, Q, info) for group g's shifted submatrix K[R, R] - mu I."""
    blk, cp, ri, gp, gb = _bsc_args(s)
    vals = _f64(s.values if values is None else values)
    mu = s.mu if mu is None else mu
    n_g, m_g = group_dims(s)
    n, m = int(n_g[g]), int(m_g[g])
    cols = np.ascontiguousarray(gb[gp[g]:gp[g + 1]], dtype=np.int32)
    rows = np.zeros(max(s.nblk, 1), dtype=np.int32)
    lam = np.zeros(n)
    q = np.zeros(n * n)
    gi = GroupInfo()
    st = lib().oracle_group_eig(s.nblk, _p(blk, ctypes.c_int32), _p(cp, ctypes.c_int64),
                                _p(ri, ctypes.c_int32), _p(vals, ctypes.c_double), len(cols),
                                _p(cols, ctypes.c_int32), float(mu), _p(rows, ctypes.c_int32),
                                _p(lam, ctypes.c_double), _p(q, ctypes.c_double), ctypes.byref(gi))
    if st != 0:
        raise RuntimeError(f"oracle_group_eig failed: {st}")
    info = {f: getattr(gi, f) for f, _ in GroupInfo._fields_}
    return rows[:m].copy(), lam, q.reshape(n, n, order="F"), info


# ---------------------------------------------------------------------------
# Frozen-iteration quantities (k Newton-Schulz steps, fixed scale), computed
# from the eigendecomposition of each group's submatrix.  Algorithm 1 of the
# paper (Sec. IV-G) reads the electron count off stored decompositions with
# signum(lambda - mu); here the signum is replaced by the k-step
# Newton-Schulz polynomial p_k of the scaled eigenvalue, which is what a
# frozen iteration evaluates.
# ---------------------------------------------------------------------------

def ns_poly(x, k):
    """p_k(x): k steps of p(x) = x (3 - x^2) / 2 (Sec. II-B) applied to scalars."""
    x = np.asarray(x, dtype=np.float64).copy()
    for _ in range(int(k)):
        x = 1.5 * x - 0.5 * x ** 3
    return x


def pade_poly(x, k):
    """k steps of the third-order Pade sign map p(x) = x (15 - 10 x^2 + 3 x^4) / 8
    (Sec. VI-A) applied to scalars."""
    x = np.asarray(x, dtype=np.float64).copy()
    for _ in range(int(k)):
        x2 = x * x
        x = x * (15.0 - 10.0 * x2 + 3.0 * x2 * x2) / 8.0
    return x


def ns_poly_deriv(x, k):
    """p_k'(x) by the chain rule through the k steps: prod (3/2)(1 - x_i^2)."""
    x = np.asarray(x, dtype=np.float64).copy()
    d = np.ones_like(x)
    for _ in range(int(k)):
        d = d * (1.5 - 1.5 * x ** 2)
        x = 1.5 * x - 0.5 * x ** 3
    return d


class GroupSpectra:
    """Eigenpairs of every group's unshifted submatrix K[R(g), R(g)] and the
    own-column weights w_gl = sum_{c in own(g)} Q_cl^2 of Algorithm 1."""

    def __init__(self, s, groups=None, values=None, nthreads=1):
        self.groups = list(range(s.ngroups)) if groups is None else list(groups)
        self.lam, self.w, self.q, self.rows = [], [], [], []
        if nthreads > 1:
            # independent groups; the C calls release the GIL
            from concurrent.futures import ThreadPoolExecutor
            with ThreadPoolExecutor(nthreads) as ex:
                eigs = list(ex.map(lambda g: group_eig(s, g, mu=0.0, values=values), self.groups))
        else:
            eigs = [group_eig(s, g, mu=0.0, values=values) for g in self.groups]
        for g, (rows, lam, q, _) in zip(self.groups, eigs):
            sizes = s.blk_size[rows]
            off = np.concatenate([[0], np.cumsum(sizes)])
            pos = {int(b): off[t] for t, b in enumerate(rows)}
            own = np.concatenate([np.arange(pos[int(j)], pos[int(j)] + s.blk_size[j])
                                  for j in s.grp_blocks[s.grp_ptr[g]:s.grp_ptr[g + 1]]])
            self.lam.append(lam)
            self.q.append(q)
            self.rows.append(rows)
            self.w.append((q[own, :] ** 2).sum(axis=0))

    def n_frozen(self, mu, k, scale):
        """N_k(mu) = sum_g sum_l w_gl (1 - p_k((lam_gl - mu)/s_g)) / 2."""
        tot = 0.0
        for t in range(len(self.groups)):
            x = (self.lam[t] - mu) / scale[t]
            tot += float((self.w[t] * 0.5 * (1.0 - ns_poly(x, k[t]))).sum())
        return tot

    def dn_dmu_frozen(self, mu, k, scale):
        """dN_k/dmu = sum_g sum_l w_gl p_k'((lam_gl - mu)/s_g) / (2 s_g)."""
        tot = 0.0
        for t in range(len(self.groups)):
            x = (self.lam[t] - mu) / scale[t]
            tot += float((self.w[t] * 0.5 * ns_poly_deriv(x, k[t]) / scale[t]).sum())
        return tot


def ns_divided_differences(x, k):
    """Matrix of divided differences (p_k(x_j) - p_k(x_l)) / (x_j - x_l) of the
    k-step polynomial, p_k'(x_j) on the diagonal.  Through one step of
    p(u) = u (3 - u^2)/2 the divided difference is 3/2 - (u^2 + u v + v^2)/2
    exactly, so the product over the steps has no cancellation."""
    u = np.asarray(x, dtype=np.float64)[:, None] * np.ones((1, len(x)))
    v = u.T.copy()
    d = np.ones_like(u)
    for _ in range(int(k)):
        d *= 1.5 - 0.5 * (u * u + u * v + v * v)
        u = 1.5 * u - 0.5 * u ** 3
        v = 1.5 * v - 0.5 * v ** 3
    return d


def frozen_gradient(s, k, scale, mu, gE=0.0, gN=0.0, gD=None, values=None):
    """Frozen map D = (I - p_k(A_g / s_g))/2 (own columns, K's layout), its N and
    E = Tr(DK), and the gradient of L = gE E + gN N + <gD, D> with respect to
    every stored value of K and to mu, by the Daleckii-Krein formula
    dL/dA_g = Q (Gamma o (Q^T W Q)) Q^T, Gamma_jl = divided differences of
    f(lam) = (1 - p_k(lam / s_g))/2 (Higham, Functions of Matrices, Thm 3.11),
    W = dL/dD_g at the own-column stored positions."""
    vals = s.values if values is None else np.asarray(values, dtype=np.float64)
    voff = s.val_off()
    d_out = np.zeros_like(vals)
    dk = np.zeros_like(vals)
    dmu = 0.0
    nblk = s.nblk
    stored = {}
    for j in range(nblk):
        for p in range(s.col_ptr[j], s.col_ptr[j + 1]):
            stored[(int(s.row_idx[p]), j)] = p
    per_group = []
    for g in range(s.ngroups):
        rows, lam, q, _ = group_eig(s, g, mu=mu, values=vals)
        sizes = s.blk_size[rows]
        off = np.concatenate([[0], np.cumsum(sizes)])
        pos = {int(b): int(off[t]) for t, b in enumerate(rows)}
        x = lam / scale[g]
        f = 0.5 * (1.0 - ns_poly(x, k[g]))
        dg = (q * f) @ q.T
        per_group.append((rows, pos, lam, q, dg))
        for j in s.grp_blocks[s.grp_ptr[g]:s.grp_ptr[g + 1]]:
            j = int(j)
            bj = s.blk_size[j]
            for p in range(s.col_ptr[j], s.col_ptr[j + 1]):
                i = int(s.row_idx[p])
                bi = s.blk_size[i]
                blk = dg[pos[i]:pos[i] + bi, pos[j]:pos[j] + bj]
                d_out[voff[p]:voff[p + 1]] = blk.reshape(-1, order="F")
    n_e = 0.0
    for j in range(nblk):
        p = stored[(j, j)]
        b = s.blk_size[j]
        n_e += np.trace(d_out[voff[p]:voff[p + 1]].reshape(b, b, order="F"))
    energy = float(np.dot(d_out, vals))
    gdl = gE * vals.copy()
    for j in range(nblk):
        p = stored[(j, j)]
        b = s.blk_size[j]
        blk = gdl[voff[p]:voff[p + 1]].reshape(b, b, order="F")
        blk[np.arange(b), np.arange(b)] += gN
        gdl[voff[p]:voff[p + 1]] = blk.reshape(-1, order="F")
    if gD is not None:
        gdl = gdl + np.asarray(gD, dtype=np.float64)
    for g in range(s.ngroups):
        rows, pos, lam, q, dg = per_group[g]
        n = q.shape[0]
        w = np.zeros((n, n))
        for j in s.grp_blocks[s.grp_ptr[g]:s.grp_ptr[g + 1]]:
            j = int(j)
            bj = s.blk_size[j]
            for p in range(s.col_ptr[j], s.col_ptr[j + 1]):
                i = int(s.row_idx[p])
                bi = s.blk_size[i]
                w[pos[i]:pos[i] + bi, pos[j]:pos[j] + bj] = gdl[voff[p]:voff[p + 1]].reshape(bi, bj, order="F")
        gamma = -0.5 * ns_divided_differences(lam / scale[g], k[g]) / scale[g]
        ga = q @ (gamma * (q.T @ w @ q)) @ q.T          # dL/dA_g
        dmu -= np.trace(ga)
        for a in rows:
            for b in rows:
                p = stored.get((int(a), int(b)))
                if p is None:
                    continue
                ba, bb = s.blk_size[a], s.blk_size[b]
                dk[voff[p]:voff[p + 1]] += ga[pos[int(a)]:pos[int(a)] + ba, pos[int(b)]:pos[int(b)] + bb].reshape(-1, order="F")
    dk += gE * d_out
    return dict(d_values=d_out, n_elec=n_e, energy=energy, dk=dk, dmu=dmu)


def symmetric_part(s, dk):
    """dK_IJ + dK_JI^T for every stored block: what symmetric changes of K see."""
    voff = s.val_off()
    where = {}
    for j in range(s.nblk):
        for p in range(s.col_ptr[j], s.col_ptr[j + 1]):
            where[(int(s.row_idx[p]), j)] = p
    out = np.empty_like(dk)
    for (i, j), p in where.items():
        q = where[(j, i)]
        bi, bj = s.blk_size[i], s.blk_size[j]
        a = dk[voff[p]:voff[p + 1]].reshape(bi, bj, order="F")
        b = dk[voff[q]:voff[q + 1]].reshape(bj, bi, order="F")
        out[voff[p]:voff[p + 1]] = (a + b.T).reshape(-1, order="F")
    return out


# ---------------------------------------------------------------------------
# Splitting submatrices into sub-submatrices (Sec. IV-C, "Splitting up
# submatrices"): the dense submatrix of a block column may still be sparse
# element by element, so the submatrix method is applied to it a second time,
# column by column, and only for the columns the block column owns.  For own
# column c of A_g = K[R, R] - mu I the sub-submatrix keeps the rows r of A_g
# whose element (r, c) is non-zero -- here |K_rc| > eps, plus r = c -- and
# D's column c is the matching column of the density of that sub-submatrix
# (zero at the rows it drops).  Plain loops and the Jacobi density above, for
# small cases only.
# ---------------------------------------------------------------------------

def split_submatrix(s, eps: float, mu: float | None = None, kT: float = 0.0, which=None) -> OracleResult:
    """D of the sub-submatrix method (K's layout; NaN outside the processed
    groups' columns), N = Tr D and E = Tr(DK) over the processed columns."""
    mu = s.mu if mu is None else mu
    vals = _f64(s.values)
    boff = np.concatenate([[0], np.cumsum(np.asarray(s.blk_size, dtype=np.int64))])
    voff = s.val_off()
    # stored blocks: (block row, block col) -> storage position
    where = {}
    for j in range(s.nblk):
        for p in range(int(s.col_ptr[j]), int(s.col_ptr[j + 1])):
            where[(int(s.row_idx[p]), j)] = p
    groups = range(s.ngroups) if which is None else [int(g) for g in which]
    d = np.full(vals.shape, np.nan)
    n_e = e_e = 0.0
    for g in groups:
        cols = [int(b) for b in s.grp_blocks[s.grp_ptr[g]:s.grp_ptr[g + 1]]]
        # step 1: R(g), the block rows stored in any of the group's block columns
        rblk = sorted({int(i) for j in cols for i in s.row_idx[s.col_ptr[j]:s.col_ptr[j + 1]]})
        rows = np.concatenate([np.arange(boff[i], boff[i + 1]) for i in rblk])
        loc = {int(r): t for t, r in enumerate(rows)}
        n = len(rows)
        # step 2: the dense submatrix A_g = K[R, R] - mu I, and which of its
        # elements lie in stored blocks
        a = np.zeros((n, n))
        stored = np.zeros((n, n), dtype=bool)
        for bi in rblk:
            for bj in rblk:
                p = where.get((bi, bj))
                if p is None:
                    continue
                blk = vals[voff[p]:voff[p + 1]].reshape(s.blk_size[bi], s.blk_size[bj], order="F")
                r0, c0 = loc[int(boff[bi])], loc[int(boff[bj])]
                a[r0:r0 + blk.shape[0], c0:c0 + blk.shape[1]] = blk
                stored[r0:r0 + blk.shape[0], c0:c0 + blk.shape[1]] = True
        a_k = a.copy()
        a -= mu * np.eye(n)
        # step 3: one sub-submatrix per own column
        for j in cols:
            for c in range(int(boff[j]), int(boff[j + 1])):
                lc = loc[c]
                keep = [r for r in range(n) if r == lc or (stored[r, lc] and abs(a_k[r, lc]) > eps)]
                sub = a[np.ix_(keep, keep)]
                dsub = dense_density(sub, kT)
                dcol = np.zeros(n)
                dcol[keep] = dsub[:, keep.index(lc)]
                # write column c of every stored block (I, j) of the block column
                for p in range(int(s.col_ptr[j]), int(s.col_ptr[j + 1])):
                    i = int(s.row_idx[p])
                    bi = int(s.blk_size[i])
                    r0 = loc[int(boff[i])]
                    cc = c - int(boff[j])
                    d[voff[p] + cc * bi:voff[p] + (cc + 1) * bi] = dcol[r0:r0 + bi]
                    e_e += float(dcol[r0:r0 + bi] @ vals[voff[p] + cc * bi:voff[p] + (cc + 1) * bi])
                n_e += float(dcol[lc])
    return OracleResult(d, n_e, e_e, [], np.asarray(list(groups), dtype=np.int32))
