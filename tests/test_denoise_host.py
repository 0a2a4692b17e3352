"""Host logic of the denoiser's comparison at equal wall time (no GPU)."""


def test_equal_time_helpers():
    import paper_2407_20692_amd.denoise_pipeline as dp
    a, b = dp.fit_linear([500, 1000, 5000], [1.5, 2.0, 6.0])
    assert abs(a - 1.0) < 1e-12 and abs(b - 1e-3) < 1e-15
    assert dp.equal_time_frames(3.0, 1.0, 1e-3, 500, 50000) == 2000
    assert dp.equal_time_frames(0.5, 1.0, 1e-3, 500, 50000) == 500
    assert dp.equal_time_frames(1e9, 1.0, 1e-3, 500, 50000) == 50000
