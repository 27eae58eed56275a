"""Pins of the 8-bit min-max table quantisation oracle (Sec. 4.3)."""
import numpy as np

from oracle import compress_oracle as QO


def _table(seed, L=3, T=64, scale=1e-1):
    g = np.random.default_rng(seed)
    return (g.uniform(-scale, scale, size=(L, T, 2)) * g.uniform(0.1, 1.0, size=(L, 1, 1))).astype(np.float32)


def test_extremes_map_to_end_codes():
    t = _table(1)
    codes, qp = QO.quantize_table(t)
    for lev in range(t.shape[0]):
        assert codes[lev].reshape(-1)[np.argmin(t[lev])] == 0
        assert codes[lev].reshape(-1)[np.argmax(t[lev])] == 255
        assert qp[lev, 0] == t[lev].min()


def test_decode_error_within_half_a_step():
    t = _table(2, L=4, T=1000)
    codes, qp = QO.quantize_table(t)
    d = QO.dequantize_table(codes, qp)
    for lev in range(4):
        step = float(qp[lev, 1])
        err = np.abs(d[lev] - t[lev].astype(np.float64)).max()
        # half a step, plus the float32 roundings of step and of (x - min) / step
        assert err <= 0.5 * step * (1 + 1e-5) + 1e-6 * step, (lev, err, step)


def test_codes_are_monotone_in_the_value():
    t = _table(3, L=2, T=500)
    codes, _ = QO.quantize_table(t)
    for lev in range(2):
        x = t[lev].reshape(-1)
        c = codes[lev].reshape(-1).astype(int)
        o = np.argsort(x, kind="stable")
        assert np.all(np.diff(c[o]) >= 0)


def test_grid_values_are_exact():
    """Values k / 256 (k = 0..255): min 0, max 255/256, step exactly 1/256,
    so every value is its own code and decodes without error."""
    k = np.arange(256, dtype=np.float32)
    t = np.stack([k / 256, k[::-1] / 256], axis=-1)[None].astype(np.float32)
    codes, qp = QO.quantize_table(t)
    assert qp[0, 0] == 0.0 and qp[0, 1] == np.float32(1 / 256)
    assert np.array_equal(codes[0, :, 0], k.astype(np.uint8))
    assert np.array_equal(QO.dequantize_table(codes, qp), t.astype(np.float64))


def test_constant_level_has_zero_step():
    t = np.full((2, 16, 2), 0.25, dtype=np.float32)
    t[1] = _table(4, L=1, T=16)[0]
    codes, qp = QO.quantize_table(t)
    assert qp[0, 1] == 0.0 and not codes[0].any()
    assert np.array_equal(QO.dequantize_table(codes, qp)[0], t[0].astype(np.float64))


def test_round_half_to_even_at_exact_midpoints():
    """min 0, max 255 -> step 1: x = k + 0.5 lies exactly between two codes
    and rounds to the even one."""
    x = np.array([0.0, 255.0, 2.5, 3.5, 100.5, 7.25], dtype=np.float32)
    t = np.stack([x, x], axis=-1)[None]
    codes, qp = QO.quantize_table(t)
    assert qp[0, 1] == 1.0
    assert list(codes[0, :, 0]) == [0, 255, 2, 4, 100, 7]
