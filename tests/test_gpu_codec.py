"""The 16-bit storages' encoder (rlb_encode16) against round-to-nearest-even
written out on the CPU, bit for bit.

Inputs: every binary32 upper half (sign, exponent and the 7 mantissa bits that
bfloat16 keeps) combined with the lower halves that decide the rounding (0,
the smallest, just below half, exactly half, just above half, the largest),
plus a seeded sample of random patterns; for binary16 also values around its
subnormal and overflow thresholds.  NaN inputs must give a NaN of the same
sign.
"""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

RLB_F16DEV, RLB_BF16DEV = 3, 4
LOW_HALVES = [0x0000, 0x0001, 0x7FFF, 0x8000, 0x8001, 0xFFFF]


def patterns() -> np.ndarray:
    hi = np.arange(1 << 16, dtype=np.uint32) << 16
    u = (hi[:, None] | np.array(LOW_HALVES, dtype=np.uint32)[None, :]).reshape(-1)
    rnd = np.random.default_rng(12).integers(0, 1 << 32, size=1 << 20, dtype=np.uint64)
    return np.concatenate([u, rnd.astype(np.uint32)])


def encode(storage: int, u: np.ndarray) -> np.ndarray:
    from paper_0912_2913_amd import _lib

    src = torch.from_numpy(u.view(np.float32).copy()).cuda()
    dst = torch.empty(u.size, dtype=torch.int16, device="cuda")
    _lib.check(_lib.lib().rlb_encode16(storage, ctypes.c_void_p(src.data_ptr()),
                                       ctypes.c_void_p(dst.data_ptr()), u.size, None),
               "rlb_encode16")
    torch.cuda.synchronize()
    return dst.cpu().numpy().view(np.uint16)


def is_nan32(u):
    return ((u & 0x7F800000) == 0x7F800000) & ((u & 0x007FFFFF) != 0)


def test_bf16_encoder_rounds_to_nearest_even():
    u = patterns()
    got = encode(RLB_BF16DEV, u).astype(np.uint32)
    nan = is_nan32(u)
    # round to nearest, ties to even, on the discarded 16 bits (carry may
    # run into the exponent: the largest finite values round to infinity)
    want = ((u.astype(np.uint64) + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint32)
    assert np.array_equal(got[~nan], want[~nan])
    g = got[nan] << 16
    assert is_nan32(g).all() and np.array_equal(g >> 31, u[nan] >> 31)


def test_fp16_encoder_rounds_to_nearest_even():
    u = patterns()
    # around binary16's subnormal range and its overflow threshold
    edge = np.float32(np.concatenate([np.linspace(-7e-8, 7e-8, 4097),
                                      np.linspace(65504.0, 65536.0, 4097),
                                      -np.linspace(65504.0, 65536.0, 4097)])).view(np.uint32)
    u = np.concatenate([u, edge])
    got = encode(RLB_F16DEV, u)
    nan = is_nan32(u)
    with np.errstate(over="ignore"):
        want = u.view(np.float32).astype(np.float16).view(np.uint16)  # IEEE conversion, RNE
    assert np.array_equal(got[~nan], want[~nan])
    g = got[nan]
    assert (((g & 0x7C00) == 0x7C00) & ((g & 0x03FF) != 0)).all()
    assert np.array_equal(g >> 15, (u[nan] >> 31).astype(np.uint16))


def test_encoder_rejects_bad_arguments():
    from paper_0912_2913_amd import _lib

    L = _lib.lib()
    buf = torch.empty(4, dtype=torch.float32, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    assert L.rlb_encode16(1, p, p, 4, None) == _lib.RLB_EINVAL  # FP32 storage
    assert L.rlb_encode16(RLB_BF16DEV, p, p, -1, None) == _lib.RLB_EINVAL
    assert L.rlb_encode16(RLB_BF16DEV, None, p, 4, None) == _lib.RLB_EINVAL
    assert L.rlb_encode16(RLB_BF16DEV, None, None, 0, None) == _lib.RLB_OK
