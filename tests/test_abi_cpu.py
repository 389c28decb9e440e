"""Host-side checks of the C-ABI library: it loads without a GPU, exports
every function include/wdr.h declares, and the binding fails loudly when
the library is missing."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wdr.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wdr_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("wdr_ctx_create", "wdr_apply_D", "wdr_apply_Dblock", "wdr_apply_schur", "wdr_solve",
              "wdr_logdet_ratio", "wdr_noise", "wdr_interpolate"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1112_1243_amd import wdr
    lib = wdr.lib()           # loads on a machine without a GPU
    for n in declared():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", wdr.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (wdr_\w+)", out))
    assert set(declared()) <= exported


def test_struct_sizes_match_the_header():
    """Compile a probe against wdr.h and compare sizeof/offsetof with ctypes."""
    from paper_1112_1243_amd import wdr
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "wdr.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu ", sizeof(wdr_geom), sizeof(wdr_solver_params),
         sizeof(wdr_solve_info), sizeof(wdr_est_params), offsetof(wdr_solver_params, tol),
         offsetof(wdr_est_params, sp), offsetof(wdr_solver_params, inner), offsetof(wdr_est_params, max_batch),
         sizeof(wdr_proposal), offsetof(wdr_proposal, kappa), offsetof(wdr_proposal, seed));
  printf("%zu %zu %zu %zu %zu %zu\n", offsetof(wdr_solver_params, block_mr_steps), offsetof(wdr_solver_params, graph),
         sizeof(wdr_solver_params), offsetof(wdr_filter_info, log_ratio), sizeof(wdr_filter_info),
         offsetof(wdr_solver_params, middle));
  return 0;
}'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "probe")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        vals = [int(v) for v in subprocess.check_output([exe]).split()]
    want = [ctypes.sizeof(wdr.Geom), ctypes.sizeof(wdr.SolverParams), ctypes.sizeof(wdr.SolveInfo),
            ctypes.sizeof(wdr.EstParams), wdr.SolverParams.tol.offset, wdr.EstParams.sp.offset,
            wdr.SolverParams.inner.offset, wdr.EstParams.max_batch.offset, ctypes.sizeof(wdr.Proposal),
            wdr.Proposal.kappa.offset, wdr.Proposal.seed.offset, wdr.SolverParams.block_mr_steps.offset,
            wdr.SolverParams.graph.offset, ctypes.sizeof(wdr.SolverParams), wdr.FilterInfo.log_ratio.offset,
            ctypes.sizeof(wdr.FilterInfo), wdr.SolverParams.middle.offset]
    assert vals == want


def test_default_params_from_library():
    from paper_1112_1243_amd import wdr
    p = wdr.default_params()
    assert p.restart == 16 and p.sap_cycles == 4 and p.mr_steps == 5 and p.tol == 1e-10
    assert p.block_mr_steps == 16 and p.update_every == 4 and p.graph == 1
    assert p.inner == wdr.F32 and p.middle == wdr.F64


def test_missing_library_raises(monkeypatch):
    from paper_1112_1243_amd import wdr
    monkeypatch.setattr(wdr, "_lib", None)
    monkeypatch.setattr(wdr, "LIB_PATH", "/nonexistent/libwdr.so")
    with pytest.raises(RuntimeError, match="not built"):
        wdr.lib()
