"""Pins of the oracle's scoring-row formats (bfloat16, FP8 E4M3 + row scale)
against the formats' definitions, hand-worked values and the library
conversions of PyTorch (CPU)."""

import numpy as np
import pytest
import torch

from oracle import quantize as Q


def test_e4m3_table_matches_definition_values():
    codes, vals = Q.e4m3_table()
    assert len(vals) == 127
    assert vals[0] == 0.0
    assert vals[1] == 2.0 ** -9                    # smallest subnormal: 1/8 * 2^-6
    assert vals[8] == 2.0 ** -6                    # smallest normal
    assert vals[0x38] == 1.0                       # exponent field 7 = bias
    assert vals[0x7E] == 448.0                     # largest finite
    assert np.all(np.diff(vals) > 0)               # monotone in the code
    assert np.isnan(Q.e4m3_value(0x7F)) and np.isnan(Q.e4m3_value(0xFF))
    assert Q.e4m3_value(0xB8) == -1.0


def test_e4m3_decode_matches_torch():
    t = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).float().numpy()
    mine = np.array([Q.e4m3_value(c) for c in range(256)])
    assert np.array_equal(np.isnan(t), np.isnan(mine))
    assert np.array_equal(t[~np.isnan(t)], mine[~np.isnan(mine)])


def test_e4m3_encode_worked_values():
    x = np.array([0.0, 1.0, 1.0625, 1.1875, 448.0, 460.0, 1e6, -3.0, 2.0 ** -10,
                  3 * 2.0 ** -10, -2.0 ** -11], dtype=np.float32)
    # 1.0625 is halfway between 1.0 (code 0x38, even) and 1.125 (0x39): even
    # 1.1875 is halfway between 1.125 (0x39) and 1.25 (0x3a): even -> 0x3a
    # 460 is nearer to 448 than to anything above; 1e6 saturates at 448
    # -3 = -1.5 * 2^1: exponent field 8, mantissa 4 -> 0xc4
    # 2^-10 is halfway between 0 and 2^-9: even code 0; 3*2^-10 -> 2^-9 * 2 (0x02)
    # -2^-11 rounds to negative zero (0x80)
    want = [0x00, 0x38, 0x38, 0x3A, 0x7E, 0x7E, 0x7E, 0xC4, 0x00, 0x02, 0x80]
    assert Q.e4m3_codes(x).tolist() == want


def test_e4m3_encode_matches_torch_in_range():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(20000) * 40, rng.standard_normal(20000) * 0.01])
    x = x.astype(np.float32)
    x = x[np.abs(x) <= 448]
    t = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(t, Q.e4m3_codes(x))


def test_bf16_round_to_nearest_even():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: even (1.0); 1 + 3*2^-8 -> up
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 3.0e38], dtype=np.float32)
    got = Q.bf16_bits(x)
    assert got[0] == 0x3F80 and got[1] == 0x3F80 and got[2] == 0x3F82
    assert Q.bf16_value(got)[3] == -2.5


def test_bf16_matches_torch():
    rng = np.random.default_rng(7)
    x = (rng.standard_normal(50000) * rng.lognormal(0, 3, 50000)).astype(np.float32)
    t = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(t, Q.bf16_bits(x))


def test_fp8_rows_scale_and_zero_row():
    x = np.array([[1.0, -2.0, 0.5], [0.0, 0.0, 0.0]], dtype=np.float32)
    codes, s = Q.fp8_rows(x)
    assert s[0] == np.float32(2.0) / np.float32(448.0) and s[1] == 0.0
    assert codes[1].tolist() == [0, 0, 0]
    assert codes[0, 1] == 0xFE                    # -448: largest magnitude, negative
    dec = np.array([Q.e4m3_value(int(c)) for c in codes[0]]) * s[0]
    assert np.allclose(dec, x[0], rtol=2 ** -3)
