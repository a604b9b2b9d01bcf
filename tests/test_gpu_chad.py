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
