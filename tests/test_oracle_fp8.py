"""FP8 E4M3 encoding (OCP 8-bit floating point, E4M3: bias 7, three mantissa bits, no
infinities, largest finite 448; round to nearest even, saturating): the oracle's
encoder against hand-computed codes, the decode/encode round trip of every code and
torch's float8_e4m3fn cast; then the library's host encoder (the one that encodes the
FP8 weights) against the oracle's.  CPU only."""
import os

import numpy as np
import pytest
import torch

import oracle as O
import paper_1709_05418_amd as ds


def sweep():
    """Every 31st float32 bit pattern with magnitude in [2^-12, 2^9], both signs, plus
    the exact subnormal, tie and saturation points."""
    u = np.arange(0x39800000, 0x44000000, 31, dtype=np.uint32)
    x = u.view(np.float32)
    ties = [O.e4m3_value(c) + (O.e4m3_value(c + 1) - O.e4m3_value(c)) / 2 for c in range(126)]
    special = np.array(ties + [O.e4m3_value(c) for c in range(127)]
                       + [448, 449, 463.99, 464, 464.01, 480, 1e6, 3.4e38, 2.0 ** -10,
                          2.0 ** -12, 1e-30, 0.0], dtype=np.float32)
    x = np.concatenate([x, special])
    return np.concatenate([x, -x])


def test_hand_computed_codes():
    cases = {0.0: 0x00, 1.0: 0x38, 448.0: 0x7E, 2.0 ** -9: 0x01, 2.0 ** -6: 0x08,
             1.0625: 0x38,    # halfway 1 and 1.125: to the even code
             1.1875: 0x3A,    # halfway 1.125 and 1.25: to the even code
             2.0 ** -10: 0x00,  # halfway 0 and 2^-9
             3 * 2.0 ** -11: 0x01, 0.875 * 2.0 ** -6: 0x07, 240.0: 0x77, -2.0: 0xC0,
             464.0: 0x7E, 1e9: 0x7E, -1e9: 0xFE}
    for v, code in cases.items():
        assert int(O.e4m3_encode(v)) == code, (v, hex(code), hex(int(O.e4m3_encode(v))))
    assert int(O.e4m3_encode(float("nan"))) == 0x7F


def test_every_code_round_trips():
    for c in range(127):
        v = O.e4m3_value(c)
        assert int(O.e4m3_encode(v)) == c
        if c:
            assert int(O.e4m3_encode(-v)) == c | 0x80
    vals = [O.e4m3_value(c) for c in range(127)]
    assert vals == sorted(vals) and vals[-1] == 448.0 and vals[1] == 2.0 ** -9


def test_matches_torch_cast_below_saturation():
    x = sweep()
    keep = np.abs(x) < 464  # torch's cast is round to nearest even without saturation
    got = O.e4m3_encode(x[keep])
    ref = torch.from_numpy(x[keep]).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(got, ref), np.nonzero(got != ref)[0][:10]
    sat = O.e4m3_encode(x[~keep])
    assert np.all((sat & 0x7F) == 0x7E)


@pytest.mark.skipif(not os.path.exists(ds.LIB_PATH), reason="libdeepscatter.so not built")
@pytest.mark.parametrize("e", [0, 3, -5, 12])
def test_library_host_encoder_matches_oracle(e):
    x = sweep()
    got = ds.ds_fp8_e4m3_encode(x, e)
    ref = O.e4m3_encode(x.astype(np.float64) * 2.0 ** e)
    assert np.array_equal(got, ref), np.nonzero(got != ref)[0][:10]
    nan = ds.ds_fp8_e4m3_encode(np.array([np.nan], np.float32))
    assert int(nan[0]) == 0x7F
