"""The CHAD coupling loop (paper_2311_08927_amd.chad) on the GPU: a few
intervals of the digester field with each reaction scheme and diffusion on;
every particle advances, the tank gas flows are positive and finite, the
particles stay in the tank, and the loop is repeatable bit for bit."""
from __future__ import annotations

import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("scheme", ["adaptive", "fixed"])
def test_loop_runs_and_repeats(torch_cuda, scheme):
    from paper_2311_08927_amd import chad
    from paper_2311_08927_amd import workloads as W
    runs = []
    for _ in range(2):
        loop = chad.Loop(8192, scheme=scheme, substeps=900, diffusion=1e-9)
        X0 = loop.X.clone()
        ch4 = []
        for _ in range(3):
            loop.interval()
            torch_cuda.cuda.synchronize()
            assert int((loop.status & 0x7F).count_nonzero()) == 0
            tot = loop.tot.cpu().numpy()
            assert np.all(np.isfinite(tot)) and tot[2] > 0.0
            ch4.append(tot[2])
        p = loop.pos.cpu().numpy()[:, :loop.n]
        assert np.all(p[0] ** 2 + p[1] ** 2 <= (W.TANK_R * (1 + 1e-6)) ** 2)
        assert np.all((p[2] >= 0) & (p[2] <= W.TANK_H))
        assert not torch_cuda.equal(loop.X, X0)
        runs.append((loop.X.clone(), ch4))
        loop.close()
    assert torch_cuda.equal(runs[0][0], runs[1][0])
    assert runs[0][1] == runs[1][1]
    print(f"{scheme}: tank CH4 flow per interval {[f'{v:.4e}' for v in runs[0][1]]}")
    assert all(math.isfinite(v) for v in runs[0][1])


@pytest.mark.parametrize("scheme", ["fixed", "adaptive"])
def test_resume_from_a_snapshot(torch_cuda, scheme, tmp_path):
    """Two intervals, a snapshot, a fresh loop resumed from it and one more
    interval: the same positions as three uninterrupted intervals, bit for
    bit, and the same states to within the solver tolerances (the S_H+
    warm starts, and the adaptive scheme's step sizes, restart from their
    defaults)."""
    from paper_2311_08927_amd import chad
    from paper_2311_08927_amd import workloads as W
    n = 8192

    def make():
        return chad.Loop(n, scheme=scheme, substeps=900, diffusion=1e-9)

    ref = make()
    for _ in range(3):
        ref.interval()
    a = make()
    for _ in range(2):
        a.interval()
    path = str(tmp_path / "chad.bin")
    a.save(path, 2 * a.dt * 86400.0)
    b = make()
    assert b.load(path) == 2 * a.dt * 86400.0
    b.interval()
    torch_cuda.cuda.synchronize()
    assert torch_cuda.equal(b.pos[:, :n], ref.pos[:, :n])
    Xb, Xr = b.X[:, :n].cpu().numpy(), ref.X[:, :n].cpu().numpy()
    scale = np.maximum(np.abs(Xr), 1e-4 * W.nominal()["state"][:, None])
    err = float((np.abs(Xb - Xr) / scale).max())
    print(f"{scheme} resume: max relative difference {err:.2e}")
    assert err < (1e-6 if scheme == "fixed" else 1e-5)
    for lp in (ref, a, b):
        lp.close()
    with pytest.raises(ValueError):
        small = chad.Loop(4096, scheme=scheme, substeps=900)
        try:
            small.load(path)
        finally:
            small.close()
