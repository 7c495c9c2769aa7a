"""FP64 CPU oracle for guided-filter non-blind deconvolution (Yang, Zhu, Zhang, Huang).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library never
calls it and shares no code with it.

Everything here is plain NumPy in float64 / complex128, written step by step from
the paper; each function names the passage it follows.  The 2-D DFT is the one
library primitive used (``numpy.fft``); everything around it is spelled out.

Readings of passages that are silent or ambiguous (periodic boundaries, the
discretised gradient, Parseval normalisation, the lambda bracket, the tie at the
infinite-lambda branch, ...) are stated next to the code that takes them.

The hand-written reverse mode of the unrolled iteration (gradients with respect to
eps and the per-iteration lambda scales) is in ``oracle.adjoint``; the boundary variants
(clipped guided-filter windows, padded non-circular observations) and their reverse mode
are in ``oracle.boundary``.

Parity status: every function here is pinned by CPU tests against closed forms,
brute force or invariants, except the multi-iteration trajectory, which has no
closed form; its parity is pinned only through its components and invariants.
The adjoint is pinned by central differences of the forward map and by an
independent float64 autograd of the same forward.
"""
from .gfd import (  # noqa: F401
    dft2, idft2, embed_psf, grad_symbol, rho_eq12, Setup, setup, residual_energy,
    discrepancy_lambda, spectral_solve, box_mean, guided_filter, guided_filter_color, StepResult, step,
    deconvolve, isnr, FLAG_INF_BRANCH, FLAG_NO_ROOT,
)
from . import adjoint  # noqa: F401,E402
from . import boundary  # noqa: F401,E402
