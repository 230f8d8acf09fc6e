"""GPU: the hand-written adjoint of the frozen Newton-Schulz map.

L = gE E + gN N + <gD, D>.  Only symmetric changes of K are meaningful, so
gradients are compared through their symmetric part dK_IJ + dK_JI^T (what
every symmetric direction sees).  Bars:
  * vs the oracle's Daleckii-Krein gradient (same k_g, s_g): 1e-9 absolute
    (FP64 iterates and adjoint; entries are O(1));
  * vs central differences (h = 1e-6, FP64, k_g and s_g frozen) on 20 random
    symmetric block directions of the 256-molecule system:
    |FD - AD| <= 1e-5 max(1, |AD|) (FD rounding ~ u |E| / h ~ 1e-7);
  * reverse dN/dmu vs the forward tangent: 1e-10 relative.
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


def sym_direction(s, rng, i, j):
    voff = s.val_off()
    where = {}
    for jj in range(s.nblk):
        for p in range(s.col_ptr[jj], s.col_ptr[jj + 1]):
            where[(int(s.row_idx[p]), jj)] = p
    bi, bj = s.blk_size[i], s.blk_size[j]
    m = rng.normal(size=(bi, bj))
    if i == j:
        m = m + m.T
    v = np.zeros_like(s.values)
    p = where[(i, j)]
    v[voff[p]:voff[p + 1]] = m.reshape(-1, order="F")
    if i != j:
        q = where[(j, i)]
        v[voff[q]:voff[q + 1]] = m.T.reshape(-1, order="F")
    return v


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16x2"])
@pytest.mark.parametrize("which", ["water16", "ragged"])
def test_backward_matches_oracle_gradient(smx, oracle_lib, which, precision):
    """The adjoint after a forward in any precision mode differentiates the
    frozen FP64 map of that evaluation (its step counts k_g, bulk plus polish,
    and scales s_g); the oracle evaluates the same map by Daleckii-Krein.  The
    explicit term gE D of E = Tr(DK) uses the evaluated D, which after a
    reduced-precision forward differs from the frozen map's D by up to 1e-6:
    the symmetric gradient then differs from the oracle's by exactly gE times
    the symmetric part of D - D_frozen (checked to 1e-9 beside it); dL/dmu has
    no explicit term and matches to 1e-9 in every mode."""
    if which == "water16":
        s = water_config("water16")
    else:
        s = random_block_system(61, [5, 3, 8, 2, 6, 4, 7, 13, 5, 5], density=0.5, coupling=0.05,
                                groups=[[0, 1], [2], [3, 4, 5], [6], [7, 8, 9]], mu=0.02)
    rng = np.random.default_rng(7)
    gd = rng.normal(size=s.values.shape)
    ge, gn = 1.0, 0.5
    ctx = smx.Context(0).load(s).configure(precision=precision)
    res = ctx.evaluate()
    info = ctx.group_info()
    dk, dmu = ctx.backward(ge, gn, gd)
    ctx.close()
    ref = oracle_lib.frozen_gradient(s, info["iters"], info["scale"], s.mu, ge, gn, gd)
    a = oracle_lib.symmetric_part(s, dk)
    b = oracle_lib.symmetric_part(s, ref["dk"])
    err = np.abs(a - b).max()
    derr = np.abs(res.d_values - ref["d_values"]).max()
    print(f"{which} {precision} forward: max|sym(dK) gpu - oracle| = {err:.2e} (max |dK| {np.abs(b).max():.2e}); "
          f"dL/dmu gpu {dmu:.10e} oracle {ref['dmu']:.10e}; max|D - D_frozen| = {derr:.1e}; "
          f"k_g {info['iters'].min()}-{info['iters'].max()}")
    explicit = ge * oracle_lib.symmetric_part(s, res.d_values - ref["d_values"])
    err_map = np.abs(a - explicit - b).max()
    print(f"  after removing gE (D - D_frozen): {err_map:.2e}")
    assert err_map <= 1e-9
    assert err <= 1e-9 + 2 * abs(ge) * derr
    assert abs(dmu - ref["dmu"]) <= 1e-9 * max(1.0, abs(ref["dmu"]))
    assert derr <= (1e-10 if precision == "fp64" else 1e-6)


def test_reverse_dn_dmu_equals_forward_tangent(smx):
    s = water_config("water16")
    ctx = smx.Context(0).load(s).configure(precision="fp64", max_iter=7, mu=0.02)
    ctx.evaluate(allow_not_converged=True)
    smx.smx_set_frozen(ctx.handle, True)
    ctx.evaluate()
    tangent = smx.smx_dn_dmu(ctx.handle)
    _, reverse = ctx.backward(0.0, 1.0)
    ctx.close()
    print(f"dN/dmu tangent {tangent:.12e} reverse {reverse:.12e}")
    assert abs(tangent - reverse) <= 1e-10 * abs(tangent)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_backward_finite_differences_water256(smx, precision):
    """Config of the differentiation run: 256 molecules, 6 A cutoff, forward in
    FP32 (FP64 polish) as the run specifies, and in FP64.  The gradient is that
    of the frozen map of the forward evaluation; the finite differences
    evaluate that frozen map (FP64, same k_g and s_g)."""
    s = water_config("water256")
    ctx = smx.Context(0).load(s).configure(precision=precision)
    ctx.evaluate()
    dk, _ = ctx.backward(1.0, 0.0)
    smx.smx_set_frozen(ctx.handle, True)
    ctx.configure(precision="fp64")
    rng = np.random.default_rng(2024)
    h = 1e-6
    worst = 0.0
    pairs = []
    while len(pairs) < 20:
        j = int(rng.integers(s.nblk))
        col = s.row_idx[s.col_ptr[j]:s.col_ptr[j + 1]]
        i = int(col[rng.integers(len(col))])
        pairs.append((i, j))
    for (i, j) in pairs:
        v = sym_direction(s, rng, i, j)
        smx.smx_update_values(ctx.handle, s.values + h * v)
        ep = ctx.evaluate().energy
        smx.smx_update_values(ctx.handle, s.values - h * v)
        em = ctx.evaluate().energy
        fd = (ep - em) / (2 * h)
        ad = float(np.dot(dk, v))
        worst = max(worst, abs(fd - ad) / max(1.0, abs(ad)))
        assert abs(fd - ad) <= 1e-5 * max(1.0, abs(ad)), (i, j, fd, ad)
    ctx.close()
    print(f"water256 dE/dK ({precision} forward): 20 symmetric block directions, "
          f"worst |FD - AD| / max(1, |AD|) = {worst:.2e}")


def test_torch_autograd_function(smx):
    torch = pytest.importorskip("torch")
    s = water_config("water16")
    ctx = smx.Context(0, stream=torch.cuda.current_stream().cuda_stream).load(s)
    f = smx.SubmatrixSign(ctx)
    k = torch.from_numpy(s.values).cuda().requires_grad_(True)
    mu = torch.tensor(0.01, dtype=torch.float64, requires_grad=True)
    d, n, e = f(k, mu)
    (e + 0.25 * n).backward()
    dk_ref, dmu_ref = ctx.backward(1.0, 0.25)
    ctx.close()
    assert np.abs(k.grad.cpu().numpy() - dk_ref).max() <= 1e-12
    assert abs(mu.grad.item() - dmu_ref) <= 1e-12 * max(1.0, abs(dmu_ref))
