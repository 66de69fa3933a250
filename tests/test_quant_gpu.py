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
