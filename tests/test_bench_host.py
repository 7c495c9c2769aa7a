"""Host logic of the benchmark (no GPU): the one-GPU contract and the byte counts its roofline
fractions divide by."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def schedule_bytes(P, Q, K, c):
    """The reverse mode's schedule walked event by event: the checkpointing replay of the first
    segments, then per segment (last first) its replays and its adjoints."""
    replay, gf, gf_save, copy = 12 * P + 76 * Q, 12 * P, 28 * P, 8 * P
    adjoint = (44 + 36) * P + (8 * P + 48 * Q) + 52 * Q + 52 * Q + (8 * P + 16 * Q)
    nck = (K + c - 1) // c
    events = [copy]                                   # starting estimate into the replay buffer
    for k in range((nck - 1) * c):
        if k % c == 0:
            events.append(copy)                       # checkpoint of the pre-estimate of k
        events += [replay, gf]
    events.append(copy)                               # checkpoint of the last segment
    for j in reversed(range(nck)):
        a, z = j * c, min(j * c + c, K)
        if j != nck - 1:
            events.append(copy)                       # checkpoint back into the replay buffer
        for _ in range(a, z):
            events += [replay, gf_save]
        events += [adjoint] * (z - a)
    return sum(events)


@pytest.mark.parametrize("K,c", [(10, 5), (7, 2), (7, 3), (1, 5), (12, 12), (13, 4)])
def test_backward_bytes_follow_the_schedule(K, c):
    P, Q = 96 * 80, 96 * 41
    assert bench.backward_bytes(P, Q, K, c) == schedule_bytes(P, Q, K, c)


def test_backward_bytes_per_pixel_iteration_at_4096():
    P, Q = 4096 * 4096, 4096 * 2049
    per = bench.backward_bytes(P, Q, 10, 5) / (P * 10)
    assert abs(per - 292.27) < 0.01
    # the forward iteration's 72 B per pixel: 4P + 8Q, 36Q, 36Q, 8P + 16Q, 12P over P
    assert abs(bench.iteration_bytes(P, Q) / P - 72.02) < 0.01
