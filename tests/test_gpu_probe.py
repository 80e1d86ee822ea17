"""The FP64 FMA probe (include/gvof_probe.h): its result is exact for a = b = 1,
and its measured rate is a plausible fraction of the chip's vector FP64 peak."""
import numpy as np
import pytest

from tests.gpu_common import host, log, torch_dev

pytestmark = pytest.mark.gpu


def test_fma_probe_result_exact():
    from paper_2111_01524_amd import probe
    torch, dev = torch_dev()
    for blocks, iters in ((1, 0), (3, 5), (37, 1001)):
        log(f"fma probe blocks={blocks} iters={iters}")
        out = torch.full((blocks * 256,), -1.0, dtype=torch.float64, device=dev)
        probe.fp64_fma(out, blocks, iters)
        torch.cuda.synchronize()
        t = np.arange(blocks * 256)
        assert np.array_equal(host(out), 28.0 + 8.0 * (t % 7) + 8.0 * iters)


def test_fma_probe_rate():
    from paper_2111_01524_amd import probe
    _, dev = torch_dev()
    tf = probe.measure_fp64_fma(dev, blocks=8192, iters=1024, repeats=3)
    log(f"fma probe {tf:.1f} TFLOP/s")
    # the published vector FP64 peak is 78.6 TFLOP/s; a loop of independent
    # FMAs at full occupancy reaches a large part of it
    assert 20.0 < tf < 90.0
