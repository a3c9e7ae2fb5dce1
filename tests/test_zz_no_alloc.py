"""The allocation-free entry point cube_get_power_noalloc against cube_get_power, through the C ABI:
two calls in a row on one GPU, the second on a smaller mesh (fewer shells), so that sums left in
the library's fixed array by the first call would show in the second."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_power_noalloc_matches_get_power():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_06121_amd import Sim
    big = synth.WORKLOADS["c1_pm32"]
    small = dict(big, np_side=32, nm_side=32, nc_side=8, box=50.0, seed=7)
    for cfg, steps in ((big, 6), (small, 4)):
        with Sim(**cfg) as sim:
            sim.init_ic()
            sim.step(steps)
            k0, p0, n0 = sim.get_power()
            nb = cfg["nm_side"] // 2
            out = [torch.full((nb,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(3)]
            sim.get_power_noalloc(*out)
            torch.cuda.synchronize()
            k1, p1, n1 = (t.cpu().numpy() for t in out)
        assert np.array_equal(n1, n0), cfg["nm_side"]
        # FP64 shell sums accumulated with atomics: equal up to the order of the additions
        assert np.allclose(k1, k0, rtol=1e-13, atol=0), cfg["nm_side"]
        assert np.allclose(p1, p0, rtol=1e-12, atol=0), cfg["nm_side"]
        assert np.all(n0 > 0) and np.all(p0 > 0)
