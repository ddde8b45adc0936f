"""Host-side logic of bench.py (no GPU): the one-GPU guard, the algorithmic
byte counts the roofline divides by, and the rule that recorded hardware
byte counts are used only while the kernel sources match their hash."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_byte_counts_at_the_bench_size():
    """M = 65536, R = 3, L = 2^17: every array read or written once, 8 bytes
    per real and 16 per complex value."""
    M, R, L = 65536, 3, 1 << 17
    vec, fac, spec, packed = 8 * M, 8 * M * R, 16 * L * R, 8 * L
    rb = bench.rhs_bytes(M, R, L)
    assert rb["phase_a"] == vec + 2 * fac + spec             # y, U, V -> spectra
    assert rb["phase_b"] == spec + packed                     # spectra -> packed input
    assert rb["phase_c"] == packed + vec + fac + vec          # packed, y, U -> S
    assert rb["rhs"] == rb["phase_a"] + rb["phase_b"] + rb["phase_c"]
    sb = bench.step_bytes(M, R, L)
    assert sb["int_a"] == 3 * vec + 2 * fac + spec            # n, k1, y2; U, V; spectra
    assert sb["int_b"] == rb["phase_b"]
    assert sb["int_c_fused"] == packed + 6 * vec + 2 * fac + spec  # y, n, k1, k2, k3, y4
    assert sb["int_c_last"] == packed + 8 * vec + fac          # n_new, n, 5 stages, k7; U
    assert set(bench.STEP_LAUNCHES) == set(sb)
    assert bench.STEP_LAUNCHES["int_b"] == 6  # one row-pair pass per DP5 right-hand side
    # compulsory bytes: n, U, V read once, S written; 4 MiB at this size
    assert bench.min_bytes(M, R) == vec + 2 * fac + vec == 4 * 2 ** 20


def test_recorded_traffic_follows_the_source_hash(monkeypatch):
    got = bench.recorded_traffic("int_c_fused")
    text = open(bench.TRAFFIC_FILE).read()
    if f"source hash: `{bench.kernel_source_hash()}`" in text:
        assert isinstance(got, int) and got > 0
    else:
        assert got is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.recorded_traffic("int_c_fused") is None
    assert bench.recorded_traffic("phase_a") is None


def test_transform_length_rule():
    """The transform length bench.py prices a size at: the smallest power of
    two >= 2 M - 2 (two length-(M-1) inputs convolve without wrap-around),
    at least 2^6, as the library chooses it."""
    for M, L in [(1, 64), (2, 64), (33, 64), (34, 128), (4096, 8192), (4097, 8192),
                 (4098, 16384), (65536, 1 << 17), (65537, 1 << 17), (65538, 1 << 18),
                 ((1 << 19) + 1, 1 << 20)]:
        assert bench.fft_length(M) == L, M
    for M in range(2, 3000):
        L = bench.fft_length(M)
        assert L >= 2 * M - 2 and (L == 64 or L // 2 < 2 * M - 2)
