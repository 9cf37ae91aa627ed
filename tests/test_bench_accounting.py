"""The benchmark's roofline accounting against hand-computed values (CPU).

Row and column passes of the 2048^2 db8 q = 2 workload: algorithmic bytes
(inputs and outputs once each, the 16-bit sample positions and the int64
offsets per (row, phase)) and algorithmic flops (2 (2 nu - 1) + log2 M per
output sample); MI355X's published FP32 vector peak and this build's issue
ceiling without packed FP32; the whole pair's minimal-traffic bytes.
"""
import bench


def test_roofline_peak():
    assert bench.VALU_PEAK_TFLOPS == 157.3
    # 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
    assert abs(bench.VALU_ISSUE_TFLOPS - 78.6432) < 1e-9
    assert bench.HBM_PEAK_GBS == 8000.0


def test_pair_bytes_2048_db8_q2():
    # per direction: x 16.8 MB, y 33.6 MB, bitmask 8.4 MB, intermediate written and read 134.2 MB
    w = dict(dim=2, j=11, q=2, nu=8)
    M, N, m, s = 2048, 8192, 8388608, 4
    fwd = M * M * s + m * s + N * N // 8 + 2 * M * N * s
    assert fwd == 192937984
    assert bench.pair_bytes(w, m, s) == 2 * fwd


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
