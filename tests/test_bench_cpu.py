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


def test_trace_summary_covers_the_timed_stencil():
    """The kernel-trace summary holds the 32^4 FP64 block-staged stencil whose
    launches the roofline object reports, with the HIP-event time beside it."""
    text = open(os.path.join(ROOT, "profiles", "estimate_wilson8_dd16_kernel_trace.md")).read()
    rows = [l for l in text.splitlines() if "k_dslash_blk<double, 4, 0, 0>" in l and "1048576x1x1" in l]
    assert rows, "no 32^4 FP64 k_dslash_blk row"
    avg_us = float(rows[0].strip().strip("|").split("|")[3])
    assert 150.0 < avg_us < 300.0
    assert "bench.py's own HIP" in text
