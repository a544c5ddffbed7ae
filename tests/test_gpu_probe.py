"""Matrix-core rate probe: it runs, its outputs are finite, and the rates it
reports are those of a working matrix core (loose bounds: the clock under load
varies from box to box)."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    yield


@pytest.mark.parametrize("kind_name,iters,lo", [("fp64", 4000, 20.0), ("int8", 8000, 1000.0),
                                               ("int8_random", 8000, 1000.0)])
def test_probe_rate(kind_name, iters, lo):
    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import mfma_probe
    kind = {"fp64": N.HSB_PROBE_FP64, "int8": N.HSB_PROBE_INT8, "int8_random": N.HSB_PROBE_INT8_RANDOM}[kind_name]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    blocks = 8 * cus
    ops, buf = mfma_probe(kind, blocks, 16)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ops, buf = mfma_probe(kind, blocks, iters, buf)
    e1.record()
    torch.cuda.synchronize()
    rate = ops / (e0.elapsed_time(e1) * 1e-3) / 1e12
    per = 16 * 16 * 4 * 2 if kind_name == "fp64" else 32 * 32 * 32 * 2
    assert ops == blocks * 4 * 4 * iters * per
    vals = buf.view(torch.float64 if kind_name == "fp64" else torch.int32)
    if kind_name == "fp64":
        assert bool(torch.isfinite(vals).all()) and bool((vals > 0).all())
    elif kind_name == "int8":
        assert bool((vals >= 0).all())
    else:  # wrapping sums of random products: not all equal
        assert int(torch.unique(vals).numel()) > 1
    print("%s probe: %.1f T ops/s" % (kind_name, rate))
    assert rate > lo
