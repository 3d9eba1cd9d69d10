"""The GPU factor generator reproduces the oracle's Gaussian stream bit for bit."""
import numpy as np
import pytest
import torch

from oracle import rng
from tests.gpu_common import banner, need_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed,draw,sketch,f,inst,rows,cols", [
    (2507, 0, 0, 1, 0, 64, 13),
    (1, 7, 3, 2, 0, 333, 17),
    (123456789012345, 4294967295, 0xFFFF, 0xFFFF, 255, 50, 40),
    (0, 0, 1, 0, 9, 1000, 33),
])
def test_gaussian_bit_exact(seed, draw, sketch, f, inst, rows, cols):
    need_gpu()
    import paper_2507_23207_amd as krp
    banner(f"gaussian seed={seed} draw={draw} sketch={sketch} f={f} inst={inst} {rows}x{cols}")
    ref = rng.factor(seed, draw, sketch, f, rows, cols, inst)  # rows x cols
    ref_cm = ref.reshape(-1, order="F")
    g64 = krp.gaussian(seed, draw, sketch, f, inst, rows, cols, "fp64").cpu().numpy()
    assert np.array_equal(g64.view(np.uint64), ref_cm.view(np.uint64))
    g32 = krp.gaussian(seed, draw, sketch, f, inst, rows, cols, "fp32").cpu().numpy()
    assert np.array_equal(g32, ref_cm.astype(np.float32))
    b16 = krp.gaussian(seed, draw, sketch, f, inst, rows, cols, "bf16").cpu().numpy().view(np.uint16)
    assert np.array_equal(b16, rng.to_bf16_bits(rng.round_fp32(ref_cm)))
    b3 = krp.gaussian(seed, draw, sketch, f, inst, rows, cols, "bf16x3").cpu().numpy().view(np.uint16)
    hi, lo = rng.split_bf16(ref_cm)
    n = rows * cols
    assert np.array_equal(b3[:n], rng.to_bf16_bits(hi))
    assert np.array_equal(b3[n:], rng.to_bf16_bits(lo))


def test_gaussian_large_stream_bit_exact():
    """One million entries: every one identical to the oracle's double."""
    need_gpu()
    import paper_2507_23207_amd as krp
    banner("gaussian 1M entries")
    rows, cols = 20000, 50
    ref = rng.factor(99, 3, 2, 1, rows, cols, 0).reshape(-1, order="F")
    g = krp.gaussian(99, 3, 2, 1, 0, rows, cols, "fp64").cpu().numpy()
    assert np.array_equal(g.view(np.uint64), ref.view(np.uint64))
