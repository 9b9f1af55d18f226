"""The allocation-free road transform (fixed device buffer) against the
workspace entry point, through the C ABI: bitwise equal fits and transformed
maps on two calls in a row, the second on a smaller frame."""
import ctypes
import math

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_1904_06017_amd.api")
from paper_1904_06017_amd._lib import RoadFit  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rolled_map(W, H, psi, seed):
    rng = np.random.default_rng(seed)
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    d = 20 + 0.11 * (v * math.cos(psi) - u * math.sin(psi)) + rng.normal(0, 0.25, (H, W))
    d[rng.uniform(size=d.shape) < 0.05] = np.nan
    mask = (rng.uniform(size=d.shape) < 0.9).astype(np.uint8)
    return d.astype(np.float32), mask


@pytest.mark.parametrize("use_mask", [True, False])
def test_noalloc_road_transform_matches_workspace_entry(use_mask):
    dev = torch.device("cuda:0")
    for (W, H, psi, seed) in ((1280, 720, 0.09, 601), (320, 240, -0.13, 602)):
        print(f"[no-alloc] road transform {W}x{H} mask={use_mask}", flush=True)
        d, m = _rolled_map(W, H, psi, seed)
        disp = torch.from_numpy(d).to(dev)
        mask = torch.from_numpy(m).to(dev) if use_mask else None
        plan = api.Plan(api.make_params(W, H, 16))
        fit_a, out_a = api.road_transform(plan, disp, mask, psi_init=0.01, delta_t=1.5)
        fit_buf = torch.zeros(ctypes.sizeof(RoadFit), dtype=torch.uint8, device=dev)
        out_b = torch.full_like(disp, -7.0)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated(dev)
        fit_b, out_b = api.road_transform_noalloc(plan, disp, mask, psi_init=0.01, delta_t=1.5,
                                                  fit_buf=fit_buf, out=out_b)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated(dev) == before
        for k in fit_a:
            if isinstance(fit_a[k], (list, tuple)):
                assert list(fit_a[k]) == list(fit_b[k]), k
            else:
                assert fit_a[k] == fit_b[k], k
        assert torch.equal(torch.isnan(out_a), torch.isnan(out_b))
        fin = ~torch.isnan(out_a)
        assert torch.equal(out_a[fin], out_b[fin])
        assert fit_b["converged"] and abs(fit_b["psi"] - psi) < 2e-3
