"""The compute roof of the cell kernels measured on the device: the vector
FMA microbenchmark of the library (vc_device_fma_rate) against the
published MI355X vector peaks (FP64 78.6 TFLOP/s; FP32 157.3 TFLOP/s with
packed instructions, half of it without, as this library is built)."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def v():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_11606_amd import vorohip
    return vorohip


def test_fma_rate_near_published_peak(v):
    fp64 = v.vc_device_fma_rate(v.VC_FP64, reps=3)
    fp32 = v.vc_device_fma_rate(v.VC_F32_FILTER, reps=3)
    print(f"measured FMA rate: FP64 {fp64:.1f} TFLOP/s, FP32 unpacked {fp32:.1f} TFLOP/s", flush=True)
    assert 0.6 * 78.6 < fp64 < 1.05 * 78.6
    assert 0.6 * 78.6 < fp32 < 1.05 * 157.3 / 2


def test_fma_rate_argument_errors(v):
    with pytest.raises(v.VcError) as e:
        v.vc_device_fma_rate(7)
    assert e.value.code == v.VC_E_ARG
    with pytest.raises(v.VcError):
        v.vc_device_fma_rate(v.VC_FP64, reps=0)
