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
