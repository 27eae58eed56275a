"""CPU oracle of the compressed-model hash tables (Sec. 4.3: the hash tables
stored with 8-bit min-max quantisation; entropy coding is a file format on
top and plays no part in rendering).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg call this module; the product path never imports it, and
this module imports nothing from the product.

Readings of what the paper leaves open:
  * min and max are taken per level of each table, over both features of
    every entry; the 256 codes span [min, max] evenly:
    step = (max - min) / 255, code = round((x - min) / step), decoded value
    min + step * code;
  * the code is an integer decided by floating point, so it is decided in
    float32 arithmetic (the storage precision of the tables): the
    subtraction, the division and the step are each rounded to float32 once,
    the rounding to an integer is to nearest with ties to even, and a level
    whose values are all equal (step 0) gets code 0;
  * decoding for the oracle's render is exact (float64).
"""
from __future__ import annotations

import numpy as np


def quantize_table(table: np.ndarray):
    """table: float32 [L][T][2].  Returns (codes uint8 [L][T][2],
    qparams float32 [L][2] = (min, step))."""
    t = np.asarray(table, dtype=np.float32)
    L = t.shape[0]
    codes = np.zeros(t.shape, dtype=np.uint8)
    qparams = np.zeros((L, 2), dtype=np.float32)
    for lev in range(L):
        x = t[lev]
        mn = np.float32(x.min())
        mx = np.float32(x.max())
        step = np.float32(np.float32(mx - mn) / np.float32(255.0))
        qparams[lev] = (mn, step)
        if step == np.float32(0.0):
            continue
        q = np.rint(np.float32(x - mn) / step)           # float32 subtract, divide; ties to even
        codes[lev] = np.clip(q, 0, 255).astype(np.uint8)
    return codes, qparams


def dequantize_table(codes: np.ndarray, qparams: np.ndarray) -> np.ndarray:
    """float64 [L][T][2]: min_l + step_l * code."""
    mn = qparams[:, 0].astype(np.float64)[:, None, None]
    st = qparams[:, 1].astype(np.float64)[:, None, None]
    return mn + st * codes.astype(np.float64)
