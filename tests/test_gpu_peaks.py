"""Measured device peaks (the rooflines' measured denominators) are positive
and within a plausible band of the published and unit-count figures of the
MI355X: integer VALU 39.3 Tops/s (256 CUs x 64 lanes x 2.4 GHz), HBM 8 TB/s,
dense BF16 MFMA 2.5 PFLOP/s, LDS 128 bytes per clock per CU (78.6 TB/s), L2
2 KB per clock per XCD (39.3 TB/s over 8 XCDs), which must beat HBM."""
import pytest

pytestmark = pytest.mark.gpu


def test_measured_peaks_are_plausible():
    import torch
    from paper_2110_13693_amd import wo
    assert torch.cuda.is_available()
    p = wo.wo_measure_peaks(2)
    print("peaks", p, flush=True)
    assert 0.5 * 39.3e12 < p["int_ops_per_s"] < 2.5 * 39.3e12
    assert 0.25 * 8e12 < p["hbm_read_bytes_per_s"] < 1.1 * 8e12
    assert 0.4 * 2.5e15 < p["bf16_flops_per_s"] < 1.1 * 2.5e15
    assert 0.25 * 78.6e12 < p["lds_bytes_per_s"] < 4.0 * 78.6e12
    assert 0.15 * 39.3e12 < p["l2_read_bytes_per_s"] < 1.2 * 39.3e12
    assert p["l2_read_bytes_per_s"] > p["hbm_read_bytes_per_s"]
