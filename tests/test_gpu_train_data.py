"""The surrogate trainer's device data handling through the C ABI: row
gathers, the seeded permutation, FP64 column statistics and the network's
residual statistics, each against numpy on the same data."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_gather_rows(torch_cuda):
    torch = torch_cuda
    from paper_2311_08927_amd import surrogate as S
    rng = np.random.default_rng(1)
    src = rng.standard_normal((1000, 35)).astype(np.float32)
    idx = rng.integers(-3, 1003, size=777).astype(np.int32)     # a few out of range
    d_src, d_idx = torch.from_numpy(src).cuda(), torch.from_numpy(idx).cuda()
    dst = torch.full((777, 35), 7.0, dtype=torch.float32, device="cuda")
    S.adm1_gather_rows(d_src, d_idx, dst)
    want = np.where(((idx >= 0) & (idx < 1000))[:, None], src[np.clip(idx, 0, 999)], 0.0)
    assert np.array_equal(dst.cpu().numpy(), want)
    # BF16 rows (128 B)
    xb = torch.from_numpy(rng.integers(-2**15, 2**15, size=(300, 64)).astype(np.int16)).cuda()
    ib = torch.from_numpy(rng.permutation(300)[:129].astype(np.int32)).cuda()
    ob = torch.empty((129, 64), dtype=torch.int16, device="cuda")
    S.adm1_gather_rows(xb, ib, ob)
    assert np.array_equal(ob.cpu().numpy(), xb.cpu().numpy()[ib.cpu().numpy()])


@pytest.mark.parametrize("n", [1, 2, 63, 64, 1000, (1 << 20) + 3])
def test_permutation(torch_cuda, n):
    torch = torch_cuda
    from paper_2311_08927_amd import surrogate as S
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    S.adm1_permutation(n, 12345, out)
    a = out.cpu().numpy()
    assert np.array_equal(np.sort(a), np.arange(n))
    S.adm1_permutation(n, 12345, out)
    assert np.array_equal(out.cpu().numpy(), a)               # deterministic
    if n >= 64:
        S.adm1_permutation(n, 12346, out)
        b = out.cpu().numpy()
        assert not np.array_equal(a, b)                        # seed-dependent
        assert np.mean(a == np.arange(n)) < 0.1                # not near the identity


def test_column_stats(torch_cuda):
    torch = torch_cuda
    from paper_2311_08927_amd import surrogate as S
    rng = np.random.default_rng(3)
    x = (rng.standard_normal((123457, 48)) * rng.uniform(0.1, 10, 48) +
         rng.uniform(-5, 5, 48)).astype(np.float32)
    m, sd = S.adm1_column_stats(torch.from_numpy(x).cuda(), 35, bf16=False)
    xd = x[:, :35].astype(np.float64)
    assert np.allclose(m, xd.mean(0), rtol=1e-12, atol=1e-12)
    assert np.allclose(sd, xd.std(0, ddof=1), rtol=1e-11)
    # BF16 bit patterns: the statistic of the rounded values
    bits = (x.view(np.uint32) >> 16).astype(np.uint16)
    xb = torch.from_numpy(np.ascontiguousarray(
        np.concatenate([bits, np.zeros((x.shape[0], 16), np.uint16)], 1)).view(np.int16)).cuda()
    mb, sdb = S.adm1_column_stats(xb, 38, bf16=True)
    xr = (bits.astype(np.uint32) << 16).view(np.float32)[:, :38].astype(np.float64)
    assert np.allclose(mb, xr.mean(0), rtol=1e-12, atol=1e-12)
    assert np.allclose(sdb, xr.std(0, ddof=1), rtol=1e-11)
    # bit-reproducible
    m2, sd2 = S.adm1_column_stats(torch.from_numpy(x).cuda(), 35, bf16=False)
    assert np.array_equal(m, m2) and np.array_equal(sd, sd2)


def test_residual_stats(torch_cuda):
    torch = torch_cuda
    from paper_2311_08927_amd import surrogate as S
    from paper_2311_08927_amd import workloads as W
    from paper_2311_08927_amd.adm1 import Context
    ctx = Context(64, rtol=1e-8, atol=W.atol_vector(1e-8))
    sur = S.Surrogate(ctx, 64, batch_max=256)
    rng = np.random.default_rng(5)
    params = (rng.standard_normal(S.NPARAMS) * 0.05).astype(np.float32)
    sur.set_weights(params, S.identity_norm(S.default_floor()))
    n = 5000
    xf = rng.standard_normal((n, 64)).astype(np.float32)
    xf[:, 38:] = 0.0
    bits = (xf.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)
    X = torch.from_numpy(np.ascontiguousarray(bits)).cuda()
    T = torch.from_numpy(rng.standard_normal((n, 35)).astype(np.float32)).cuda()
    mean, msq = S.adm1_surrogate_residual_stats(sur.handle, X, T, chunk=777)
    Y = sur.forward(X)[:, :35].double().cpu().numpy()
    r = Y - T.double().cpu().numpy()
    assert np.allclose(mean, r.mean(0), rtol=1e-10, atol=1e-12)
    assert np.allclose(msq, (r * r).mean(0), rtol=1e-10)
    sur.close()
    ctx.close()
