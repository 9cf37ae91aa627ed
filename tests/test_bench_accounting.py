"""The benchmark's roofline accounting against hand-computed values (CPU).

Row and column passes of the 2048^2 db8 q = 2 workload: algorithmic bytes
(inputs and outputs once each, the 16-bit sample positions and the int64
offsets per (row, phase)) and algorithmic flops (2 (2 nu - 1) + log2 M per
output sample), and the FP32 FMA peak without packed instructions.
"""
import bench


def test_roofline_peak():
    # 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
    assert abs(bench.VALU_PEAK_TFLOPS - 78.6432) < 1e-9
    assert bench.HBM_PEAK_GBS == 8000.0


def test_stage_bytes_2048_db8_q2():
    w = dict(j=11, q=2, nu=8)
    M, N, Q, m, s = 2048, 8192, 4, 8388608, 4
    b = bench.stage_bytes(w, m, s)
    omega = 2 * m + 8 * (N * Q + 1)
    assert b[("fwd", 2)] == (M * N + m) * s + omega == 117702664
    assert b[("adj", 0)] == b[("fwd", 2)]
    assert b[("fwd", 1)] == (M * M + M * N) * s == 83886080
    assert b[("adj", 1)] == b[("fwd", 1)]
    assert b[("fwd", 0)] == b[("adj", 2)] == 2 * M * M * s
    # a full Omega carries no sample list
    full = bench.stage_bytes(w, N * N, s)
    assert full[("fwd", 2)] == (M * N + N * N) * s


def test_stage_flops_2048_db8_q2():
    f = bench.stage_flops(dict(j=11, q=2, nu=8))
    per = 2 * 15 + 11
    assert f[("fwd", 2)] == f[("adj", 0)] == 8192 * 8192 * per == 2751463424
    assert f[("fwd", 1)] == f[("adj", 1)] == 2048 * 8192 * per
