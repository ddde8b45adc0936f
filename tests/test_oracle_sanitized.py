"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): the C source is built with -fsanitize=address,undefined (every
undefined-behaviour report fatal) and every entry point is driven on small
and degenerate inputs (M = 1, 2, ragged sizes, ranks 1..5, each scheme,
controller and formula kernel, the proposer functions) by a child Python
process with the ASan runtime preloaded.  Any out-of-bounds access, use of
freed memory or undefined operation ends that process with a report."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "smol_oracle.c")

DRIVER = textwrap.dedent("""
    import numpy as np
    import oracle
    import workloads as W

    for M in (1, 2, 3, 7, 64, 129):
        for R in (1, 3, 5):
            U, V = W.random_factors(M, R, seed=M + R)
            n = W.random_state(M, seed=M)
            S = oracle.rhs(U, V, 0.02, n, threads=2)
            idx = np.unique(np.array([0, M // 2, M - 1]))
            assert np.allclose(oracle.rhs_entries(U, V, 0.02, n, idx, threads=2), S[idx],
                               rtol=1e-12, atol=1e-300)
            oracle.rhs_source(U, V, 0.02, n, np.full(M, 1e-3))
        for f in (1, 2, 3):
            oracle.rhs_kernel(f, 0.01, W.random_state(M, seed=3), p0=0.4, p1=1.0)
        oracle.kernel_matrix(3, M)
    for M in (1, 2, 50):
        U, V = W.brownian_rank3(M, 1.0 / 3.0)
        n0 = W.monodisperse(M)
        for method in (oracle.BS32, oracle.DP54):
            out, st, log = oracle.integrate(U, V, 0.01, n0, 2.0, 1e-6, 1e-12, method=method,
                                            log_cap=8)
            assert st["status"] == 0, st
            oracle.integrate(U, V, 0.01, n0, 2.0, 1e-6, 1e-12, method=method, max_steps=3)
            oracle.integrate(U, V, 0.01, n0, 0.0, 1e-6, 1e-12, method=method)
            oracle.rk_fixed(U, V, 0.01, n0, method, 0.1, 3, embedded=True)
            oracle.tableau(method)
        for scheme in (oracle.RKF45, oracle.RK2_DBL, oracle.RK4_DBL):
            for rule in (oracle.RULE_EQ6, oracle.RULE_HALVE_DOUBLE, oracle.RULE_FEHLBERG):
                oracle.integrate_paper(U, V, 0.01, n0, 1.0, 1e-5, scheme, rule, log_cap=4)
            oracle.paper_attempt(U, V, 0.01, n0, 0.1, scheme)
    # the proposer: features, network, gradient, Adam, training rows, decisions
    n = W.random_state(40, seed=9)
    mom = oracle.moments(n)
    oracle.features(n, 0.1, [0.3, 0.2])
    oracle.proposer_features(mom, 0.1, [0.3, 0.2, 0.1, 0.05])
    params = W.mlp_init(seed=1)
    X = np.random.default_rng(0).standard_normal((5, 9))
    oracle.mlp_forward(params, X)
    loss, grad = oracle.mlp_loss_grad(params, X, np.zeros(5))
    m, v = np.zeros_like(params), np.zeros_like(params)
    oracle.adam(params.copy(), grad, m, v, 1)
    U, V = W.brownian_rank3(60, 0.4)
    out, st, log = oracle.integrate(U, V, 0.01, W.monodisperse(60), 5.0, 1e-6, 1e-12,
                                    log_cap=400)
    rows = np.zeros((len(log), 9))
    rows[:, :5] = log
    oracle.proposer_dataset(rows, 5)
    oracle.learned_factor(params, mom, 0.1, [0.3, 0.2, 0.1, 0.05], 0.2, 5)
    oracle.learned_steps(params, rows, 5)
    print("sanitized oracle: every entry point ran", flush=True)
""")


def _asan_runtime():
    try:
        path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                              text=True, timeout=60).stdout.strip()
    except (OSError, subprocess.SubprocessError):
        return None
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    asan = _asan_runtime()
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    so = str(tmp_path / "liboracle_sanitized.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-fPIC",
                           "-shared", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-o", so, SRC, "-lm"],
                          timeout=300)
    env = dict(os.environ, ORACLE_LIB=so, LD_PRELOAD=asan, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24",
               PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", DRIVER], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    report = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
    assert "every entry point ran" in r.stdout
