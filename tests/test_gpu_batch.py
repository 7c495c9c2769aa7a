"""Batched contexts: one context for many independent images gives, image by image, exactly
what separate single-image contexts give (same kernels and arithmetic, one launch per pass),
and matches the FP64 oracle like a single image does."""
import numpy as np
import pytest
import torch

import oracle
import paper_1609_01839_amd as gfd
import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

# mixed kinds: register-resident transforms (powers of two >= 256), LDS transforms (others)
SMALL_SIZES = [(64, 80), (96, 96), (256, 256), (75, 90), (128, 120), (256, 512), (45, 75), (512, 256)]


def to_gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def problems(cases):
    return [dict(y=to_gpu(c.y), h=to_gpu(c.h.astype(np.float32)), sigma2=c.sigma2, w=c.w, eps=c.eps) for c in cases]


def single_runs(probs, chunks, estimates=None):
    out = []
    for k, p in enumerate(probs):
        with gfd.GFDeconv(p["y"], p["h"], p["sigma2"], p["w"], p["eps"]) as g:
            if estimates is not None:
                g.set_estimate(estimates[k])
            lams = []
            for n in chunks:
                u, lam = g.iterate(n)
                lams.append(lam.cpu().numpy())
            out.append((u.cpu().numpy(), np.concatenate(lams), g.info()))
    return out


def test_batch_equals_single_contexts():
    cases = synth.make_batch(10, sizes=SMALL_SIZES)
    print("batch:", " ".join(f"{c.y.shape[0]}x{c.y.shape[1]}/w{c.w}" for c in cases))
    probs = problems(cases)
    ref = single_runs(probs, [2, 4])
    with gfd.GFDeconvBatch(probs) as g:
        us1, lam1 = g.iterate(2)
        us1 = [u.cpu().numpy() for u in us1]
        us, lam2 = g.iterate(4)
        lams = np.concatenate([lam1.cpu().numpy(), lam2.cpu().numpy()], axis=1)
        for b, (u_ref, lam_ref, info) in enumerate(ref):
            assert np.array_equal(us[b].cpu().numpy(), u_ref), b
            assert np.array_equal(lams[b], lam_ref), b
            ii = g.image_info(b)
            assert (ii["M"], ii["N"]) == u_ref.shape
            assert ii["rho"] == info["rho"] and ii["target"] == info["target"]
        assert g.info()["iterations"] == 6


def test_batch_graph_equals_eager_and_reset():
    cases = synth.make_batch(5, sizes=SMALL_SIZES, config=7)
    probs = problems(cases)
    res = []
    with gfd.GFDeconvBatch(probs) as g:
        for use_graph in (True, False):
            g.set_graph(use_graph)
            g.reset()
            us, lam = g.iterate(4)
            res.append(([u.cpu().numpy() for u in us], lam.cpu().numpy()))
    for a, b in zip(res[0][0], res[1][0]):
        assert np.array_equal(a, b)
    assert np.array_equal(res[0][1], res[1][1])


def test_batch_set_estimate_uses_concatenated_layout():
    cases = synth.make_batch(4, sizes=SMALL_SIZES, config=9)
    probs = problems(cases)
    rng = np.random.default_rng(5)
    est = [to_gpu(rng.uniform(0, 255, c.y.shape)) for c in cases]
    ref = single_runs(probs, [2], estimates=est)
    with gfd.GFDeconvBatch(probs) as g:
        g.set_estimate(est)
        us, lam = g.iterate(2)
        for b, (u_ref, lam_ref, _) in enumerate(ref):
            assert np.array_equal(us[b].cpu().numpy(), u_ref), b
            assert np.array_equal(lam.cpu().numpy()[b], lam_ref), b


def test_batch_matches_oracle():
    cases = synth.make_batch(3, sizes=[(64, 80), (96, 96), (256, 256)], config=11)
    probs = problems(cases)
    iters = 4
    with gfd.GFDeconvBatch(probs) as g:
        us, lam = g.iterate(iters)
        us = [u.cpu().numpy() for u in us]
        lam = lam.cpu().numpy()
    for b, c in enumerate(cases):
        eps = float(np.float32(c.eps))
        ref_u, info = oracle.deconvolve(c.y.astype(np.float64), c.h.astype(np.float32).astype(np.float64), c.sigma2,
                                        c.w, eps, iters)
        e = float(np.linalg.norm(us[b] - ref_u) / np.linalg.norm(ref_u))
        le = max(abs(float(lam[b, k]) - info["lam"][k]) / info["lam"][k] for k in range(iters))
        print(f"{c.name}: rel L2 {e:.2e}, lambda {le:.2e}")
        assert e < 1e-5 and le < 1e-4


def config3_mix():
    """One image of every size of the mixed-size batch workload, with each of its PSF kinds
    (the 9x9 box, whose transform has exact zeros along the 480- and 720-row axes, at 480x640
    and 720x1280), its BSNR range and its window sizes."""
    specs = [((256, 256), "gauss", 5, 24.0), ((480, 640), "box9", 7, 38.0), ((512, 512), "invq", 9, 31.0),
             ((720, 1280), "box9", 5, 20.0), ((1024, 1024), "gauss", 9, 40.0)]
    cases = []
    for k, ((M, N), kind, w, bsnr) in enumerate(specs):
        rng = np.random.default_rng(3000 + k)
        u = synth.piecewise_image(M, N, rng)
        h = {"box9": lambda: synth.psf_box(9), "gauss": lambda: synth.psf_gaussian(float(rng.uniform(1.0, 3.0)), 25),
             "invq": lambda: synth.psf_inverse_quadratic(15)}[kind]()
        b = synth.blur_periodic(u, h)
        s2 = synth.sigma2_for_bsnr(b, bsnr)
        y = (b + np.sqrt(s2) * rng.standard_normal((M, N))).astype(np.float32)
        cases.append(synth.Case(f"{M}x{N}_{kind}_w{w}", u, h, y, s2, w, synth.EPS_DEFAULT, 4))
    return cases


def test_batch_matches_oracle_every_batch_size():
    cases = config3_mix()
    iters = 4
    refs = []
    for c in cases:
        eps = float(np.float32(c.eps))
        _, info = oracle.deconvolve(c.y.astype(np.float64), c.h.astype(np.float32).astype(np.float64), c.sigma2, c.w,
                                    eps, iters, keep_iterates=True)
        refs.append(info)
    errs = np.zeros((len(cases), iters))
    lerr = np.zeros((len(cases), iters))
    with gfd.GFDeconvBatch(problems(cases)) as g:
        for k in range(iters):
            us, lam = g.iterate(1)
            lam = lam.cpu().numpy()
            for b, c in enumerate(cases):
                ref = refs[b]["iterates"][k]
                errs[b, k] = np.linalg.norm(us[b].cpu().numpy() - ref) / np.linalg.norm(ref)
                lo = refs[b]["lam"][k]
                assert np.isfinite(lo) == np.isfinite(lam[b, 0]), (b, k)
                lerr[b, k] = abs(float(lam[b, 0]) - lo) / lo if np.isfinite(lo) else 0.0
    for b, c in enumerate(cases):
        print(f"{c.name}: iterate rel L2 " + " ".join(f"{e:.1e}" for e in errs[b]) +
              f", lambda {lerr[b].max():.1e}")
    assert errs.max() < 1e-5 and lerr.max() < 1e-4


def test_batch_rejects_single_image_calls():
    cases = synth.make_batch(2, sizes=[(64, 80)], config=13)
    with gfd.GFDeconvBatch(problems(cases)) as g:
        lib = gfd.load_library()
        lam = torch.empty(1, device=DEV)
        u = torch.zeros(64 * 80, device=DEV)
        assert lib.discrepancy_lambda(g.handle, u.data_ptr(), lam.data_ptr(), None) == -5


def test_autotune_keeps_state_and_results():
    c = synth.make_case(1, size=(512, 512))
    y, h = to_gpu(c.y), to_gpu(c.h.astype(np.float32))
    with gfd.GFDeconv(y, h, c.sigma2, c.w, c.eps) as ref:
        u_ref, lam_ref = ref.iterate(5)
        u_ref, lam_ref = u_ref.cpu().numpy(), lam_ref.cpu().numpy()
    with gfd.GFDeconv(y, h, c.sigma2, c.w, c.eps) as g:
        choice = g.autotune(3)
        print("autotune choice", choice)
        assert g.info()["iterations"] == 0
        u, lam = g.iterate(5)
        u, lam = u.cpu().numpy(), lam.cpu().numpy()
        with pytest.raises(gfd.GFDError):
            g.autotune(3)              # iterations have run
    e = float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref))
    print(f"tuned vs default rel L2 {e:.2e}")
    assert e < 1e-6 and np.allclose(lam, lam_ref, rtol=1e-5)


def test_set_tuning_results():
    c = synth.make_case(1, size=(512, 512))
    y, h = to_gpu(c.y), to_gpu(c.h.astype(np.float32))
    with gfd.GFDeconv(y, h, c.sigma2, c.w, c.eps) as ref:
        u_ref, lam_ref = ref.iterate(4)
        u_ref, lam_ref = u_ref.cpu().numpy(), lam_ref.cpu().numpy()
    with gfd.GFDeconv(y, h, c.sigma2, c.w, c.eps) as g:
        with pytest.raises(gfd.GFDError):
            g.set_tuning(-1, 0, 0)
        g.set_tuning(48, 1, 2)         # strip height, forward row pairs, inverse rows
        u, lam = g.iterate(4)
        u, lam = u.cpu().numpy(), lam.cpu().numpy()
        with pytest.raises(gfd.GFDError):
            g.set_tuning(48, 1, 2)     # iterations have run
    e = float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref))
    print(f"set shapes vs default rel L2 {e:.2e}")
    assert e < 1e-6 and np.allclose(lam, lam_ref, rtol=1e-5)


def test_mixed_radix_tuning_knobs():
    """The mixed-radix transforms' knobs (rows per block of the LDS row passes, radix-4 schedule)
    change launch shapes and the order of the butterflies only: results agree with the default
    shapes to rounding and with the oracle to the iterate bar."""
    c = synth.make_case(1, size=(480, 640))
    y, h = to_gpu(c.y), to_gpu(c.h.astype(np.float32))
    iters = 4
    with gfd.GFDeconv(y, h, c.sigma2, c.w, c.eps) as ref:
        u_ref, lam_ref = (t.cpu().numpy() for t in ref.iterate(iters))
    ref_o, _ = oracle.deconvolve(c.y.astype(np.float64), c.h.astype(np.float32).astype(np.float64), c.sigma2, c.w,
                                 float(np.float32(c.eps)), iters)
    for rows, radix in ((2, 4), (8, 8), (4, 4)):
        with gfd.GFDeconv(y, h, c.sigma2, c.w, c.eps) as g:
            with pytest.raises(gfd.GFDError):
                g.set_tuning(0, 0, 0, 0, 3)    # schedules are 8 and 4
            g.set_tuning(0, 0, 0, rows, radix)
            u, lam = (t.cpu().numpy() for t in g.iterate(iters))
        e = float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref))
        eo = float(np.linalg.norm(u - ref_o) / np.linalg.norm(ref_o))
        print(f"rows {rows} radix {radix}: vs default {e:.2e}, vs oracle {eo:.2e}")
        assert e < 1e-6 and eo < 1e-5 and np.allclose(lam, lam_ref, rtol=1e-5)


@pytest.mark.skip(reason="autotuning a multi-image context ended twice in a host segmentation fault inside "
                         "the HIP runtime during its trials (this test once, the 64-image batch of bench.py "
                         "once, under rocprofv3), whose cause has not been found by reading the code; the "
                         "library now refuses it (GFD_ERR_UNIMPLEMENTED) and the case stays off the GPU")
def test_autotune_batch():
    cases = synth.make_batch(4, sizes=SMALL_SIZES, config=19)
    probs = problems(cases)
    ref = single_runs(probs, [3])
    with gfd.GFDeconvBatch(probs) as g:
        g.autotune(2)
        us, _ = g.iterate(3)
        for b, (u_ref, _, _) in enumerate(ref):
            e = float(np.linalg.norm(us[b].cpu().numpy() - u_ref) / np.linalg.norm(u_ref))
            assert e < 1e-6, (b, e)


def test_batch_autotune_refused_and_set_tuning_works():
    """A multi-image context refuses deconv_autotune (before any trial) and takes launch shapes
    from deconv_set_tuning: the tuned batch agrees with the images' own default-shape contexts
    to rounding."""
    cases = synth.make_batch(4, sizes=SMALL_SIZES, config=19)
    probs = problems(cases)
    ref = single_runs(probs, [3])
    with gfd.GFDeconvBatch(probs) as g:
        with pytest.raises(gfd.GFDError) as ei:
            g.autotune(2)
        assert ei.value.code == -6
        g.set_tuning(32, 1, 2, 2, 8)
        us, _ = g.iterate(3)
        for b, (u_ref, _, _) in enumerate(ref):
            e = float(np.linalg.norm(us[b].cpu().numpy() - u_ref) / np.linalg.norm(u_ref))
            assert e < 1e-6, (b, e)
