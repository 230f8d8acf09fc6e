"""GPU: the boundary calls around an evaluation.

* caller-owned work space (smx_workspace_size / smx_set_workspace, e.g. a
  torch tensor): results bitwise equal to the library-allocated arena, with
  one wave and with waves forced by a smaller work space; error paths;
* enqueue-only evaluation (smx_set_host_poll(0)): bitwise equal to the
  polled run;
* convergence histories (smx_get_history) against the oracle's
  eigendecomposition: X_k = Q p_k(Lambda / s) Q^T, so max|X_k^2 - I| and
  Tr(I - X_k^2) follow from the eigenpairs for every step k.
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


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


def evaluate(ctx):
    r = ctx.evaluate()
    return r.d_values.copy(), r.n_elec, r.energy, ctx.group_info()


@pytest.mark.parametrize("precision", ["fp64", "fp16x2", "bf16x3", "fp32"])
def test_torch_workspace_is_bitwise_equal(smx, torch, precision):
    s = random_block_system(71, [13, 5, 5, 17, 9, 31, 22, 13, 27, 11, 5, 25] * 2, density=0.45,
                            coupling=0.05, groups="pairs", mu=0.01)
    ctx = smx.Context(0).load(s).configure(precision=precision)
    d0, n0, e0, i0 = evaluate(ctx)
    need = smx.smx_workspace_size(ctx.handle)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    smx.smx_set_workspace(ctx.handle, ws)
    d1, n1, e1, i1 = evaluate(ctx)
    st1 = ctx.stats()
    assert st1["nwaves"] == 1
    # about half of it: the groups run in waves through the caller's memory
    half = torch.empty(need // 2 + 4096, dtype=torch.uint8, device="cuda")
    smx.smx_set_workspace(ctx.handle, half)
    d2, n2, e2, i2 = evaluate(ctx)
    st2 = ctx.stats()
    smx.smx_set_workspace(ctx.handle, None)
    d3, n3, e3, _ = evaluate(ctx)
    ctx.close()
    print(f"{precision}: work space {need / 2**20:.1f} MiB, waves with half of it: {st2['nwaves']}")
    assert st2["nwaves"] >= 2
    for d, n, e, i in ((d1, n1, e1, i1), (d2, n2, e2, i2)):
        np.testing.assert_array_equal(d, d0)
        assert n == n0 and e == e0
        np.testing.assert_array_equal(i["iters"], i0["iters"])
        np.testing.assert_array_equal(i["resid"], i0["resid"])
    np.testing.assert_array_equal(d3, d0)


def test_workspace_errors(smx, torch):
    s = water_config("water16")
    ctx = smx.Context(0).load(s)
    need = smx.smx_workspace_size(ctx.handle)
    big = torch.empty(need + 1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(smx.SmxError) as e:          # not 256-byte aligned
        smx.smx_set_workspace(ctx.handle, big.data_ptr() + 8, need)
    assert e.value.code == smx.SMX_E_INVALID
    host = np.zeros(need // 8 + 64)
    with pytest.raises(smx.SmxError) as e:          # host memory
        smx.smx_set_workspace(ctx.handle, host.ctypes.data // 256 * 256 + 256, 4096)
    assert e.value.code == smx.SMX_E_INVALID
    tiny = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    smx.smx_set_workspace(ctx.handle, tiny)
    with pytest.raises(smx.SmxError) as e:          # smaller than the largest group
        ctx.evaluate()
    assert e.value.code == smx.SMX_E_NOMEM
    smx.smx_set_workspace(ctx.handle, None)
    ctx.evaluate()
    ctx.close()


@pytest.mark.parametrize("precision,graph_steps", [("fp64", 0), ("fp16x2", 0), ("fp16x2", 4)])
def test_enqueue_only_is_bitwise_equal(smx, torch, precision, graph_steps):
    s = water_config("water16")
    ctx = smx.Context(0).load(s).configure(precision=precision, graph_steps=graph_steps)
    d0, n0, e0, i0 = evaluate(ctx)
    smx.smx_set_host_poll(ctx.handle, False)
    for _ in range(2):
        d1, n1, e1, i1 = evaluate(ctx)
        np.testing.assert_array_equal(d1, d0)
        assert n1 == n0 and e1 == e0
        np.testing.assert_array_equal(i1["iters"], i0["iters"])
    ctx.close()


def _oracle_histories(oracle_lib, s, g, scale, nsteps):
    """max|X_k^2 - I| and Tr(I - X_k^2) for k < nsteps, from the eigenpairs."""
    _, lam, q, _ = oracle_lib.group_eig(s, g)
    x = lam / scale
    res, tau = [], []
    for k in range(nsteps):
        f = 1.0 - x * x                    # eigenvalues of I - X_k^2
        res.append(float(np.abs((q * f) @ q.T).max()))
        tau.append(float(f.sum()))
        x = 1.5 * x - 0.5 * x ** 3
    return np.array(res), np.array(tau)


@pytest.mark.parametrize("precision", ["fp64", "fp16x2"])
def test_history_matches_oracle(smx, oracle_lib, precision):
    s = water_config("water16")
    ctx = smx.Context(0).load(s).configure(precision=precision)
    ctx.evaluate()
    info = ctx.group_info()
    h = smx.smx_get_history(ctx.handle, 64)
    ctx.close()
    polish = 0 if precision == "fp64" else 2
    np.testing.assert_array_equal(h["nsteps"], info["iters"] - polish + 1)
    for g in (0, 7, s.ngroups - 1):
        n = int(h["nsteps"][g])
        assert np.all(np.isnan(h["resid"][g, n:]))
        r_or, t_or = _oracle_histories(oracle_lib, s, g, info["scale"][g], n)
        r = h["resid"][g, :n]
        if precision == "fp64":
            assert np.all(np.isnan(h["tau"][g]))
            assert np.all(np.abs(r - r_or) <= 1e-11 + 1e-10 * r_or)
            assert r[-1] <= 1e-12 < r[-2]
        else:
            t = h["tau"][g, :n]
            # FP32-accumulated products of the words: ~1e-6 relative to the diagonal sums
            assert np.all(np.abs(t - t_or) <= 1e-4 + 1e-5 * t_or), (g, t, t_or)
            assert np.all(np.abs(r - r_or) <= 1e-5 + 1e-4 * r_or), (g, r, r_or)
            assert t[-1] <= 1e-3 < t[-2]
        print(f"{precision} group {g}: {n} steps, resid {r[0]:.3e} -> {r[-1]:.3e}"
              + ("" if precision == "fp64" else f", tau {h['tau'][g, 0]:.3e} -> {h['tau'][g, n - 1]:.3e}"))


@pytest.mark.parametrize("precision,npairs", [("fp64", 1), ("fp16x2", 3), ("bf16x3", 6)])
def test_launch_issued_flops_accounting(smx, precision, npairs):
    """smx_get_launch_issued on one group of n = 368 (n_pad = 384, three 128-row
    tiles): every launch that works on the group issues 21 live 64 x 64 wave tiles
    (3 x 3 in the diagonal tiles, 3 x 4 below them) of 2 x 64 x 64 x n_pad flops,
    times the word products per algorithmic product; the others issue nothing."""
    s = water_config("water16")
    one = s.with_groups([list(range(s.nblk))])
    ctx = smx.Context(0).load(one).configure(precision=precision)
    ctx.evaluate()
    ms, algo, kind = ctx.launch_profile()
    issued = smx.smx_get_launch_issued(ctx.handle)
    ctx.close()
    assert len(issued) == len(algo) > 0
    n, npad = 368, 384
    per = 21 * 2.0 * 64 * 64 * npad * npairs
    for a, q in zip(algo, issued):
        if a > 0:
            assert a == 2.0 * n ** 3 and q == per
        else:
            assert q == 0.0
