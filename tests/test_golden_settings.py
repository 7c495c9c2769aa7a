"""The synthetic workloads reproduce the degradation settings the paper prints (Table 1, Sec. 4)."""
import json
import os

import numpy as np

import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_settings.json")))


def test_table1_psfs_and_noise_levels():
    for t, spec in GOLD["tests"].items():
        kind, s2 = synth.TABLE1_SETTINGS[int(t)]
        assert s2 == spec["sigma2"]
    hq = synth.psf_inverse_quadratic(15, normalise=False)
    assert hq.shape == (15, 15) and hq[7, 7] == 1.0 and hq[0, 0] == 1.0 / (1 + 49 + 49)
    assert np.isclose(synth.psf_inverse_quadratic(15).sum(), 1.0)
    b = synth.psf_binomial()
    assert b.shape == (5, 5) and b[2, 2] == 36 / 256 and b[0, 0] == 1 / 256 and b.sum() == 1.0
    box = synth.psf_box(9)
    assert box.shape == (9, 9) and np.allclose(box, 1 / 81)
    g = synth.psf_gaussian(1.6, 25)
    assert np.isclose(g.sum(), 1.0) and g[12, 12] == g.max()
    # second moment of the sampled Gaussian matches its standard deviation
    i = np.arange(-12, 13)
    assert abs(np.sqrt(np.sum(g.sum(axis=1) * i ** 2)) - 1.6) < 1e-3


def test_paper_guided_filter_parameters_on_the_255_scale():
    c = synth.table1_case(3, 32, 32)
    assert c.w == GOLD["guided_filter"]["w"]
    assert np.isclose(c.eps, GOLD["guided_filter"]["eps_unit_scale"] * 255 ** 2)
    assert np.isclose(c.sigma2, 0.308)


def test_bsnr_noise_level():
    c = synth.make_case(1, size=(128, 128))
    blurred = synth.blur_periodic(c.u_orig, c.h)
    assert np.isclose(10 * np.log10(np.var(blurred) / c.sigma2), 40.0)
    assert c.y.dtype == np.float32
