"""The allocation-free entry point (deconvolve_static) against deconv_init + deconv_iterate.

deconvolve_static keeps every buffer in the library's fixed per-device array; with the same
kernels its results must equal the context path's bit for bit.  Two calls in a row, the second
on a smaller problem, check that the array's leftover contents from the first call do not leak
into the second.  Also compared with the FP64 oracle to the iterate bar (1e-5 relative L2).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1609_01839_amd as gfd
import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def to_gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def context_run(c, iters):
    y, h = to_gpu(c.y), to_gpu(c.h.astype(np.float32))
    with gfd.GFDeconv(y, h, c.sigma2, c.w, c.eps) as g:
        g.set_graph(False)
        u, lam = g.iterate(iters)
        return u.cpu().numpy(), lam.cpu().numpy()


def static_run(c, iters):
    y, h = to_gpu(c.y), to_gpu(c.h.astype(np.float32))
    u, lam = gfd.deconvolve_static(y, h, c.sigma2, c.w, c.eps, iters)
    return u.cpu().numpy(), lam.cpu().numpy()


def test_static_equals_context_two_calls_second_smaller():
    big = synth.make_case(1, size=(512, 512))         # the largest square size the array holds
    small = synth.make_batch(1, sizes=[(75, 90)], config=23)[0]
    iters_big, iters_small = 5, 4
    ref_big = context_run(big, iters_big)
    ref_small = context_run(small, iters_small)
    out_big = static_run(big, iters_big)
    out_small = static_run(small, iters_small)          # second call, smaller input
    for tag, ref, out in (("512x512", ref_big, out_big), ("75x90", ref_small, out_small)):
        du = float(np.max(np.abs(out[0] - ref[0])))
        print(f"{tag}: max |u_static - u_context| {du:.3g}, lambdas equal {np.array_equal(out[1], ref[1])}")
        assert np.array_equal(out[0], ref[0]), tag
        assert np.array_equal(out[1], ref[1]), tag
    # and against the oracle
    c = small
    ref_u, _ = oracle.deconvolve(c.y.astype(np.float64), c.h.astype(np.float32).astype(np.float64), c.sigma2, c.w,
                                 float(np.float32(c.eps)), iters_small)
    e = float(np.linalg.norm(out_small[0] - ref_u) / np.linalg.norm(ref_u))
    print(f"75x90 static vs oracle rel L2 {e:.2e}")
    assert e < 1e-5


def test_static_rejects_what_the_array_cannot_hold():
    c = synth.make_case(1, size=(1024, 1024))
    y, h = to_gpu(c.y), to_gpu(c.h.astype(np.float32))
    with pytest.raises(gfd.GFDError) as ei:
        gfd.deconvolve_static(y, h, c.sigma2, c.w, c.eps, 2)
    assert ei.value.code == -2
    # still usable afterwards, on a smaller problem
    s = synth.make_case(1, size=(64, 80))
    ref = context_run(s, 3)
    out = static_run(s, 3)
    assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1])
