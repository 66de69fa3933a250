"""epm_quantize against the input generator's encoders (which are pinned
against torch's CPU conversions in test_synth.py), code for code."""

import numpy as np
import pytest

import synth
from tests.gpu_util import torch_gpu

pytestmark = pytest.mark.gpu


def _rows():
    rng = np.random.default_rng(11)
    parts = [rng.normal(size=(300, 128)) * m for m in (1e-6, 1.0, 3e4)]
    special = np.zeros((4, 128))
    # scale exactly 1 (amax = 448): E4M3 ties and the subnormal range
    special[1, 0] = 448.0
    special[1, 1:9] = [1.0625, 1.1875, -1.0625, 2.0 ** -10, 3 * 2.0 ** -10, 2.0 ** -6,
                       2.0 ** -6 - 2.0 ** -10, 440.0]
    special[2] = -0.0  # an all-zero row of negative zeros: scale 1, sign kept
    special[3, :64] = 1e-30  # a tiny row: the scale follows it down
    return np.concatenate(parts + [special]).astype(np.float32)


def test_bf16_codes_equal_the_generator():
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    x = _rows()
    got = E.quantize(torch.from_numpy(x).to("cuda:0"), "bf16").cpu().numpy().view(np.uint16)
    assert np.array_equal(got, synth.f32_to_bf16(x))


def test_fp8_codes_and_scales_equal_the_generator():
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    x = _rows()
    codes, scale = E.quantize(torch.from_numpy(x).to("cuda:0"), "fp8")
    rc, rs = synth.f32_to_fp8_e4m3(x)
    assert np.array_equal(scale.cpu().numpy(), rs)
    assert np.array_equal(codes.cpu().numpy(), rc)
    # the hand-made ties: 1.0625 -> 1.0 (0x38), 1.1875 -> 1.25 (0x3A)
    c = codes.cpu().numpy()[901]
    assert c[1] == 0x38 and c[2] == 0x3A and c[3] == 0xB8
    assert np.all(codes.cpu().numpy()[902] == 0x80)


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_rounding_error_bounds_the_dequantisation_error(fmt):
    """epm_rounding_error: a bound on |x - dequant(x^)| per row, within 1e-5
    (relative) of the exact norm, never below it."""
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(41)
    x = synth.pairs._unit_rows(rng.standard_normal((3000, 128)))
    x[7] = 0.0  # an all-zero row
    if fmt == "bf16":
        codes = synth.f32_to_bf16(x)
        deq = synth.bf16_to_f32(codes).astype(np.float64)
        err = E.rounding_error(torch.from_numpy(x).to(dev),
                               torch.from_numpy(codes.view(np.int16)).to(dev), "bf16")
    else:
        codes, scale = synth.f32_to_fp8_e4m3(x)
        deq = synth.fp8_e4m3_to_f32(codes) * scale[:, None].astype(np.float64)
        err = E.rounding_error(torch.from_numpy(x).to(dev), torch.from_numpy(codes).to(dev),
                               "fp8", scale=torch.from_numpy(scale).to(dev))
    exact = np.linalg.norm(x.astype(np.float64) - deq, axis=1)
    got = err.cpu().numpy().astype(np.float64)
    assert (got >= exact).all()
    assert (got <= exact * (1 + 1e-5) + 1e-29).all()
    assert got[7] < 1e-20
