"""Host-side checks of the lambda-search state machine used by the HIP kernels.

The header is compiled for the CPU with g++; sums are exact (double) so that only the
bracketing / interpolation logic is under test.  The reference root comes from a float64
bisection of sum q (lam / (t + lam))^2 = T P, written here independently.
"""
import ctypes
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    d = tempfile.mkdtemp()
    so = os.path.join(d, "lamhost.so")
    src = os.path.join(ROOT, "tests", "host", "lam_search_driver.cpp")
    inc = os.path.join(ROOT, "paper_1609_01839_amd", "csrc")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", inc, src, "-o", so], check=True)
    l = ctypes.CDLL(so)
    l.lam_search_host.restype = ctypes.c_int
    l.lam_search_host.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_float, ctypes.c_float,
                                  ctypes.c_int, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int)]
    l.lam_rounds.restype = ctypes.c_int
    l.lam_rounds.argtypes = [ctypes.c_int]
    l.lam_search_sequence.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    return l


@pytest.fixture(scope="module")
def sweeps(lib):
    """Evaluation rounds after the first one: (per iteration, warm start / stand-alone search),
    the same constants the library compiles in."""
    return lib.lam_rounds(0), lib.lam_rounds(1)


def run(lib, q, t, TP, lam_prev=0.0, rounds=3):
    q = np.ascontiguousarray(q, np.float32)
    t = np.ascontiguousarray(t, np.float32)
    lam, used = ctypes.c_float(), ctypes.c_int()
    flags = lib.lam_search_host(q.ctypes.data, t.ctypes.data, q.size, TP, lam_prev, rounds, ctypes.byref(lam),
                                ctypes.byref(used))
    return lam.value, used.value, flags


def ref_root(q, t, TP):
    q = q.astype(np.float64)
    t = t.astype(np.float64)
    f = lambda lam: np.sum(q * (lam / (t + lam)) ** 2)
    lo, hi = 1e-30, 1e30
    for _ in range(300):
        mid = math.sqrt(lo * hi)
        if f(mid) < TP:
            lo = mid
        else:
            hi = mid
    return math.sqrt(lo * hi)


def log_slope(q, t, lam):
    """d ln f / d ln lambda at lam: FP32 evaluation errors in f reach lambda divided by this."""
    q = q.astype(np.float64)
    r = 1.0 / (1.0 + t.astype(np.float64) / lam)
    return 2.0 * np.sum(q * r * r * (1.0 - r)) / np.sum(q * r * r)


def tolerance(q, t, lam):
    return 2e-6 + 3e-8 / log_slope(q, t, lam)


def spectra(n, seed, decay):
    rng = np.random.default_rng(seed)
    t = np.exp(-decay * rng.uniform(0, 1, n) ** 2 * 20)          # |H|^2 from 1 down to tiny values
    q = rng.exponential(1.0, n) * (1.0 + 50 * t)
    return q.astype(np.float32), t.astype(np.float32)


@pytest.mark.parametrize("seed,decay,frac", [(0, 1.0, 0.3), (1, 0.5, 0.05), (2, 2.0, 0.8), (3, 1.0, 0.999),
                                             (4, 3.0, 1e-4)])
def test_cold_start_converges_within_the_launched_rounds(lib, sweeps, seed, decay, frac):
    """A cold start (no previous lambda) is what the warm-start and stand-alone searches do."""
    q, t = spectra(20000, seed, decay)
    E = float(np.sum(q.astype(np.float64)))
    TP = np.float32(frac * E)
    lam, used, flags = run(lib, q, t, float(TP), rounds=sweeps[1])
    ref = ref_root(q, t, float(TP))
    tol = tolerance(q, t, ref)
    print(f"seed {seed}: lam {lam:.8g} ref {ref:.8g} rel {abs(lam - ref) / ref:.1e} tol {tol:.1e} rounds {used}")
    assert flags == 0
    assert abs(lam - ref) / ref < tol
    assert used <= sweeps[1] + 1


@pytest.mark.parametrize("shift", [1.0, 1.3, 0.7, 4.0, 0.2])
def test_warm_start_converges_fast(lib, sweeps, shift):
    q, t = spectra(20000, 7, 1.0)
    TP = float(np.float32(0.2 * np.sum(q.astype(np.float64))))
    ref = ref_root(q, t, TP)
    lam, used, flags = run(lib, q, t, TP, lam_prev=ref * shift, rounds=sweeps[0])
    print(f"warm x{shift}: rel {abs(lam - ref) / ref:.1e} rounds {used}")
    assert flags == 0
    assert abs(lam - ref) / ref < tolerance(q, t, ref)
    assert used <= sweeps[0] + 1


def test_infinite_branch_and_no_root(lib):
    q, t = spectra(1000, 9, 1.0)
    E = float(np.sum(q.astype(np.float64)))
    lam, used, flags = run(lib, q, t, E * 1.0001)
    assert math.isinf(lam) and flags == 1
    t0 = t.copy()
    t0[:500] = 0.0                     # exact spectral zeros: f(0+) = sum of q over them
    lam, used, flags = run(lib, q, t0, float(np.sum(q[:500].astype(np.float64))) * 0.5)
    assert flags == 2 and lam == pytest.approx(1e-30)


def sequence(lib, q, t, TP, rounds):
    n = len(TP)
    lam = (ctypes.c_float * n)()
    used = (ctypes.c_int * n)()
    flags = (ctypes.c_int * n)()
    q32, t32 = np.ascontiguousarray(q, np.float32), np.ascontiguousarray(t, np.float32)
    TP = np.ascontiguousarray(TP, np.float32)
    lib.lam_search_sequence(q32.ctypes.data, t32.ctypes.data, q.size, TP.ctypes.data, n, rounds,
                            ctypes.cast(lam, ctypes.c_void_p), ctypes.cast(used, ctypes.c_void_p),
                            ctypes.cast(flags, ctypes.c_void_p))
    return list(lam), list(used), list(flags)


def test_settling_sequence_uses_two_rounds_after_the_jump(lib, sweeps):
    """Targets that move like a real iteration: a big first jump, then a slow drift, with the
    rounds an iteration launches."""
    q, t = spectra(20000, 11, 1.0)
    E = float(np.sum(q.astype(np.float64)))
    fr = [0.30, 0.05, 0.06, 0.058, 0.0585, 0.0586, 0.0586]
    TP = np.array([f * E for f in fr], np.float32)
    lam, used, flags = sequence(lib, q, t, TP, sweeps[0])
    for k in range(len(fr)):
        ref = ref_root(q, t, float(TP[k]))
        print(f"step {k}: rel {abs(lam[k] - ref) / ref:.1e} rounds {used[k]} flags {flags[k]}")
        assert abs(lam[k] - ref) / ref < tolerance(q, t, ref)
        assert flags[k] == 0
    assert max(used[4:]) <= 2          # settled: first round + at most one refinement
    assert max(used[1:]) <= sweeps[0] + 1


@pytest.mark.parametrize("jump", [0.3, 3.0, 30.0, 1e4, 1e-4])
def test_jump_past_the_first_candidates(lib, sweeps, jump):
    """After a settled sequence (first spacing at its 0.02 minimum) the target moves so far that
    the root leaves the first round's outer candidates (+-3.5 spacings): within the rounds an
    iteration launches, lambda either converges or the unconverged flag is raised."""
    q, t = spectra(20000, 13, 1.0)
    E = float(np.sum(q.astype(np.float64)))
    base = 0.05 * E
    f_jump = float(np.clip(base * (1.0 + jump) if jump > 1e-3 else base * 0.3, 1e-6 * E, 0.9 * E))
    TP = np.array([base, base, base, base, f_jump], np.float32)
    lam, used, flags = sequence(lib, q, t, TP, sweeps[0])
    ref_prev = ref_root(q, t, float(TP[3]))
    ref = ref_root(q, t, float(TP[4]))
    err = abs(lam[4] - ref) / ref
    print(f"jump x{ref / ref_prev:.3g}: rel {err:.1e} rounds {used[4]} flags {flags[4]}")
    assert abs(math.log(ref / ref_prev)) > 3.5 * 0.02
    assert used[4] <= sweeps[0] + 1
    if flags[4] & 8:
        assert used[4] == sweeps[0] + 1   # only the forced last decision raises it
    else:
        assert flags[4] == 0 and err < tolerance(q, t, ref)


def test_forced_decision_raises_the_unconverged_flag(lib):
    """With a single round after the first, a far jump from a warm start cannot converge: the
    decision forced at the round limit raises the flag."""
    q, t = spectra(20000, 17, 1.0)
    E = float(np.sum(q.astype(np.float64)))
    ref_prev = ref_root(q, t, 0.05 * E)
    lam, used, flags = run(lib, q, t, float(np.float32(0.95 * E)), lam_prev=ref_prev, rounds=1)
    print(f"rounds {used} flags {flags}")
    assert flags == 8 and used == 2
