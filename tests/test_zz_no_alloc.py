"""The allocation-free sketch entry point (krp_sketch_noalloc) against krp_sketch.

Both launch the same kernels with the same plans, so the sketches agree bit
for bit; two calls in a row (the second on a smaller tensor, so it sees the
previous call's partial sums in the shared per-GPU array) and every policy."""
import numpy as np
import pytest
import torch

from tests.gpu_common import banner, need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _ys(x, modes, ells):
    return [torch.empty((l, x.shape[m]), dtype=x.dtype, device=x.device).t() for m, l in zip(modes, ells)]


@pytest.mark.parametrize("prec,dt", [("bf16x3", torch.float32), ("fp32", torch.float32),
                                     ("fp64", torch.float64)])
def test_noalloc_matches_sketch_on_two_calls(prec, dt):
    need_gpu()
    import paper_2507_23207_amd as krp
    rs = np.random.default_rng(51)
    cases = [((96, 64, 40, 12), [0, 1, 2, 3], [24, 17, 40, 9]),   # larger first
             ((40, 33, 20), [2, 0], [11, 20])]                      # then smaller, ragged
    for dims, modes, ells in cases:
        x = to_dev(rs.standard_normal(dims), dt)
        banner(f"noalloc {prec} {dims}")
        ref = krp.sketch(x, modes, ells, prec=prec, seed=77, draw=3)
        ys = krp.sketch_noalloc(x, modes, ells, _ys(x, modes, ells), prec=prec, seed=77, draw=3)
        torch.cuda.synchronize()
        for m, a, b in zip(modes, ys, ref):
            assert torch.equal(a, b), (dims, m, float((a - b).abs().max()))
