"""Pins of the growth-map definitions (oracle/growth.py): constant and linear fields give
closed forms, the window length, the box corners of the feature map, and the bin order."""
import math

import numpy as np

from oracle import growth as Gr


def test_window_cells():
    assert Gr.window_cells(0.1) == 63          # 2 pi / 0.1 = 62.83
    assert Gr.window_cells(100.0) == 1
    assert Gr.window_cells(2 * math.pi / 10.4) == 10


def test_constant_field_growth_is_log_amplitude():
    # |E| = |B| = a S on every cell: A^2/S^2 = 2 a^2, G = ln a + ln(2)/2 everywhere
    a, S = 37.0, 1e-6
    le = np.full(50, math.log(a * S))
    G = Gr.windowed_growth(le, le, 0.5, S)
    assert np.max(np.abs(G - (math.log(a) + 0.5 * math.log(2)))) < 1e-13


def test_linear_power_window_mean():
    # A^2/S^2 = i + 1 on cell i (|B| = 0): the mean of a window of consecutive integers
    S, h = 1.0, 2 * math.pi / 4          # w = 4
    n = 12
    le = 0.5 * np.log(np.arange(1, n + 1, dtype=np.float64))
    lb = np.full(n, -np.inf)
    G = Gr.windowed_growth(le, lb, h, S)
    for j in range(n):
        lo = max(0, j - 3)
        ref = 0.5 * math.log(np.mean(np.arange(lo + 1, j + 2)))
        assert abs(G[j] - ref) < 1e-14
    # first cells: growing windows (1), (1,2), (1,2,3)
    assert abs(G[1] - 0.5 * math.log(1.5)) < 1e-15


def test_features_box_corners():
    lo = np.array([[math.log(1e-3), math.log(10.0), 0.05, 0.0, 0.0]])
    hi = np.array([[math.log(1e-1), math.log(1e4), 4.0, 200.0, 10.0 * math.sqrt(1e4 / 1e-1)]])
    assert np.allclose(Gr.features(lo), -1.0, atol=1e-14)
    assert np.allclose(Gr.features(hi), 1.0, atol=1e-14)
    assert abs(Gr.tau_final(0.01, 1000.0) - 10.0 * math.sqrt(1e5)) < 1e-9


def test_bin_order():
    x = np.array([[-1, -1, -1, -1, -1], [1, 1, 1, 1, 1], [-1, -1, -1, -1, -0.74], [-0.74, -1, -1, -1, -1]], float)
    assert list(Gr.bin_of(x)) == [0, 8 ** 5 - 1, 1, 8 ** 4]


def test_p99_table_definition():
    # 100 errors 1e-3 .. 0.1 in one bin: the 99th smallest is 0.099, whose bucket
    # (1e-4 2^(39/4), 1e-4 2^10] = (0.0861, 0.1024] reports 0.1024
    x = np.zeros((100, 5))
    err = np.arange(1, 101) * 1e-3
    t = Gr.p99_table(x, err)
    b = int(Gr.bin_of(x[:1])[0])
    assert abs(t[b] - 1e-4 * 2 ** 10) < 1e-15
    assert np.sum(t >= 0) == 1
    # fewer than 32 examples: no estimate
    assert np.all(Gr.p99_table(x[:31], err[:31]) == -1)
    # bucket edges bracket their errors
    for e in (1e-5, 1e-4, 1.0001e-4, 3e-3, 0.5, 7.0):
        bb = Gr.bucket(e)
        assert e <= Gr.bucket_edge(bb) and (bb == 0 or e > Gr.bucket_edge(bb - 1))
    assert Gr.bucket(np.inf) == Gr.bucket(np.nan) == Gr.bucket(1e30) == 63
