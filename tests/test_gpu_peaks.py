"""GPU: the measured peaks (pecnn_measure_peaks) are positive, ordered and in the range the chip's
datasheet allows; undersized or misaligned scratch is refused before any launch."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2403_12820_amd import _lib
    _lib.lib()
    return _lib


def test_measured_peaks_are_plausible(L):
    import torch
    scratch = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    pk = L.pecnn_measure_peaks(scratch)
    assert set(pk) == set(L.PEAK_KEYS)
    # datasheet: FP32 VALU 39.3e12 lane operations/s without packed math, FP64 the same, bf16 MFMA
    # 2.5e15 FLOP/s dense, FP32 MFMA 157e12; a copy this small may be served by the 256 MB cache
    assert 1e11 < pk["hbm_copy_bytes_per_s"] < 1e14
    assert 5e12 < pk["fp32_valu_fma_lane_ops_per_s"] < 4.5e13
    assert 1e11 < pk["rsq_f32_lane_ops_per_s"] < pk["fp32_valu_fma_lane_ops_per_s"]
    assert 2e12 < pk["fp64_valu_fma_lane_ops_per_s"] < 4.5e13
    assert 2e14 < pk["bf16_mfma_flop_per_s"] < 2.8e15
    assert 2e13 < pk["fp32_mfma_flop_per_s"] < 1.8e14


def test_measure_peaks_refuses_bad_scratch(L):
    import torch
    small = torch.empty(32 << 20, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.PecnnError, match="64 MiB"):
        L.pecnn_measure_peaks(small)
    big = torch.empty((64 << 20) + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.PecnnError, match="aligned"):
        L.pecnn_measure_peaks(big[16:])
