"""The oracle's own decoders of the low-precision input formats, over every
code, against torch's conversions (a library routine)."""
import numpy as np
import torch


def _same(a, b):
    return np.array_equal(np.isnan(a), np.isnan(b)) and \
        np.array_equal(a[~np.isnan(a)], b[~np.isnan(b)])


def test_bf16_all_codes(orc):
    codes = np.arange(1 << 16, dtype=np.uint16)
    mine = orc.decode_bf16(codes)
    ref = torch.from_numpy(codes.view(np.int16)).view(torch.bfloat16).double().numpy()
    assert _same(mine, ref)
    # signed zeros keep their sign
    assert np.signbit(mine[0x8000]) and not np.signbit(mine[0])


def test_e4m3_all_codes(orc):
    codes = np.arange(256, dtype=np.uint8)
    mine = orc.decode_e4m3(codes)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).double().numpy()
    assert _same(mine, ref)
    assert np.nanmax(mine) == 448.0 and np.isnan(mine[0x7f]) and np.isnan(mine[0xff])
