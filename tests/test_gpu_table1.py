"""The five settings of Table 1 (PSF, noise variance; w = 3 and eps of Sec. 4) on synthetic
stand-in images: the GPU trajectory over 30 iterations against the FP64 oracle, with rho from
Eq.(12) and with rho = 1 -- every iterate within 1e-5 relative L2, every lambda within 1e-4 and
the final ISNR within 0.01 dB."""
import numpy as np
import pytest
import torch

import oracle
import paper_1609_01839_amd as gfd
from paper_1609_01839_amd import table1
import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.mark.parametrize("rho", [None, 1.0])
@pytest.mark.parametrize("test", [1, 2, 3, 4, 5])
def test_table1_setting_matches_oracle(test, rho):
    c = synth.table1_case(test, 128, 128)
    iters = 30
    eps = float(np.float32(c.eps))
    ref_u, info = oracle.deconvolve(c.y.astype(np.float64), c.h.astype(np.float32).astype(np.float64), c.sigma2,
                                    c.w, eps, iters, rho=rho, keep_iterates=True)
    y, h = torch.from_numpy(c.y).to(DEV), torch.from_numpy(c.h.astype(np.float32)).to(DEV)
    errs, lams = [], []
    with gfd.GFDeconv(y, h, c.sigma2, c.w, eps, rho) as g:
        for k in range(iters):
            u, lam = g.iterate(1)
            errs.append(float(np.linalg.norm(u.cpu().numpy() - info["iterates"][k]) / np.linalg.norm(info["iterates"][k])))
            lams.append(float(lam.cpu()[0]))
    lam_ref = info["lam"]
    finite = np.isfinite(lam_ref)
    assert np.array_equal(np.isfinite(lams), finite)
    lam_err = float(np.max(np.abs(np.array(lams)[finite] / lam_ref[finite] - 1.0))) if finite.any() else 0.0
    ig, io = table1.isnr(u.cpu().numpy(), c.y, c.u_orig), oracle.isnr(ref_u, c.y, c.u_orig)
    print(f"test {test} rho {rho}: max iterate rel L2 {max(errs):.1e}, lambda {lam_err:.1e}, ISNR {ig:.4f}/{io:.4f} dB")
    assert max(errs) < 1e-5 and lam_err < 1e-4 and abs(ig - io) < 0.01


def test_table1_driver_runs():
    res = table1.run(size=64, iters=3, rho_choices=(None,))
    assert len(res) == 5 and all(np.isfinite(r["isnr_db"]) for r in res)
