"""The autotuner returns valid options, caches them, and the tuned options
solve the same problem to the same answer."""
import os

import numpy as np
import pytest

from paper_2009_12638_amd import inputs, ms
from gpu_util import dev, host, say, torch_cuda

pytestmark = pytest.mark.gpu


def test_autotune_valid_and_cached(tmp_path, orc):
    torch = torch_cuda()
    from paper_2009_12638_amd import tune
    shape = (64, 64, 64)
    cuts = [inputs.uniform_cuts(64, 2)] * 3
    b = dev(inputs.poisson_randn(shape, 140))
    cache = str(tmp_path / "tune.json")
    say("autotune 64^3")
    out = tune.autotune(shape, cuts, b, precision="mixed", cache=cache)
    assert out["rows"] in (1, 2, 4) and out["x_chunk"] in (8, 16, 32)
    assert out["inner_iters"] in tune.INNER_CANDIDATES
    assert os.path.exists(cache)
    again = tune.autotune(shape, cuts, b, precision="mixed", cache=cache)
    assert again == out
    # tuned tiling changes the schedule, not the arithmetic: same iterate as default
    h = ms.ms_create(shape, cuts=[list(map(int, c)) for c in cuts])
    x1 = torch.zeros(shape, dtype=torch.float64, device="cuda")
    x2 = torch.zeros_like(x1)
    ms.ms_solve(h, b, x1, 0.0, 10, "sync", max_sweeps=6, precision="mixed")
    ms.ms_solve(h, b, x2, 0.0, 10, "sync", max_sweeps=6, precision="mixed",
                rows=out["rows"], x_chunk=out["x_chunk"])
    d = float(torch.linalg.norm(x1 - x2) / torch.linalg.norm(x1))
    assert d <= 1e-5   # FP32 inner sums in a different tile order
