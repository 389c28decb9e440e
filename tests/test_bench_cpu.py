"""Host-side checks of bench.py: it refuses more than one GPU with a message,
and the committed stencil counter summary belongs to the current stencil
sources (otherwise the reported traffic would be null)."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_summary_matches_stencil_sources():
    bench = load_bench()
    for prec in ("f64", "f32", "f16"):
        t = bench.counted_traffic(prec)
        assert t is not None, "counter summary is stale for " + prec
        assert t > 0
    # FP64 moves more than its algorithmic 768 B per site at 32^4, and less than twice that
    alg = 768 * 32 ** 4
    assert alg < bench.counted_traffic("f64") < 2 * alg


def test_eo16_counter_summary_is_fresh():
    """The roofline's traffic for the dominant kernel of the headline comes
    from a counter summary of the current cg16.hip, within 1.0x-1.5x of the
    algorithmic bytes."""
    bench = load_bench()
    t = bench.counted_traffic_eo16(32)
    assert t is not None, "k_eo16 counter summary is stale"
    alg = 32 * (bench.eo16_bytes(32 ** 4, False) + bench.eo16_bytes(32 ** 4, True)) // 2
    assert alg < t < 1.5 * alg


def test_trace_summary_covers_the_headline():
    """The kernel-trace summary isolates the timed 32^4 estimates and holds
    the dominant kernel k_eo16 in the launch shape of the roofline object
    (32 systems per launch), with bench.py's own timing beside it."""
    text = open(os.path.join(ROOT, "profiles", "estimate_wilson32_dd4096_kernel_trace.md")).read()
    assert "Kernels inside the timed range" in text
    rows = [l for l in text.splitlines() if l.startswith("| k_eo16") and "524288x32x1" in l]
    assert rows, "no k_eo16 row at 32 systems per launch"
    avg_us = float(rows[0].strip().strip("|").split("|")[4])
    assert 500.0 < avg_us < 2000.0
    assert "bench.py reported" in text


def test_variance_fit_recovers_known_model():
    """fit_variance on synthetic pairs with a known law: log Rhat_N of pair q
    is g_q + e_{q,N} with g_q ~ N(0, a) shared by every N of the pair and
    independent e ~ N(0, b / N), so Var(log Rhat_N) = a + b / N.  The fit
    recovers a within four bootstrap errors, the bootstrap error is close to
    the spread of the estimate over independent repetitions, and the 68%
    interval covers the truth in about 68% of them."""
    bench = load_bench()
    import numpy as np
    a_true, b_true, Ns, P = 0.4, 20.0, (8, 16, 32, 64), 200
    rng = np.random.Generator(np.random.Philox(key=[7, 11]))
    ests, errs, cover = [], [], 0
    for rep in range(40):
        g = rng.normal(0.0, np.sqrt(a_true), P)
        lr = np.stack([g + rng.normal(0.0, np.sqrt(b_true / N), P) for N in Ns], axis=1)
        f = bench.fit_variance(lr, Ns, n_boot=300, seed=rep)
        ests.append(f["a"])
        errs.append(f["a_err"])
        cover += f["a_68"][0] <= a_true <= f["a_68"][1]
        assert abs(f["a"] - a_true) < 4 * f["a_err"] + 1e-12
        assert abs(f["b"] - b_true) < 0.5 * b_true
    spread = float(np.std(ests, ddof=1))
    assert 0.6 < float(np.mean(errs)) / spread < 1.6
    assert 16 <= cover <= 38
