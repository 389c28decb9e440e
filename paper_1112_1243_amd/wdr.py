"""Python binding of the HIP library ``libwdr.so`` (C ABI in include/wdr.h).

Argument marshalling only: every step runs in the library's kernels.
Fields are torch tensors on the GPU in the canonical layout:
  spinors  complex128 [V, 4, 3]      gauge fields  complex128 [V, 4, 3, 3]
and calls are ordered on torch's current HIP stream.  There is no CPU
fallback: if the library is missing, loading it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("WDR_LIB", os.path.join(_HERE, "libwdr.so"))

# ---------------------------------------------------------------- constants (wdr.h)
OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, ESTATE = 0, -1, -2, -3, -4, -5
F64, F32, F16 = 0, 1, 2
STENCIL_AUTO, STENCIL_DIR, STENCIL_BLK = 0, 1, 2
MR_AUTO, MR_ONE_PER_CU, MR_TWO_PER_CU = 0, 1, 2
CG_LAUNCHES, CG_PERSISTENT = 0, 1
NOISE_Z2, NOISE_GAUSS = 0, 1
OP_FULL, OP_SCHUR, OP_BLOCKS, OP_DD = 0, 1, 2, 3
SOLVER_FGCR_SAP, SOLVER_CGNE = 0, 1


class Geom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4), ("B", ctypes.c_int32 * 4), ("bc", ctypes.c_int32 * 4)]


class SolverParams(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int), ("restart", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("sap_cycles", ctypes.c_int32), ("mr_steps", ctypes.c_int32), ("tol", ctypes.c_double),
                ("block_tol", ctypes.c_double), ("adj_tol", ctypes.c_double), ("inner", ctypes.c_int),
                ("middle", ctypes.c_int), ("block_mr_steps", ctypes.c_int32), ("update_every", ctypes.c_int32),
                ("graph", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("true_rel_resid", ctypes.c_double),
                ("seconds", ctypes.c_double), ("total_iters", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FilterInfo(ctypes.Structure):
    _fields_ = [("block_accepts", ctypes.c_int32), ("block_trials", ctypes.c_int32), ("accepted", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("log_ratio", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class EstParams(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int), ("n_steps", ctypes.c_int32), ("n_noise", ctypes.c_int32),
                ("noise", ctypes.c_int), ("seed", ctypes.c_uint64), ("sp", SolverParams),
                ("max_batch", ctypes.c_int32)]


class Proposal(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("U", ctypes.c_void_p), ("Up", ctypes.c_void_p),
                ("kappa", ctypes.c_double), ("seed", ctypes.c_uint64)]


class WdrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("wdr status %d: %s" % (status, msg))
        self.status = status


_lib = None


def lib():
    """Load libwdr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is not built: run __graft_entry__.build() or "
                               "python paper_1112_1243_amd/build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, i32, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        L.wdr_last_error.restype = ctypes.c_char_p
        L.wdr_status_str.restype = ctypes.c_char_p
        L.wdr_status_str.argtypes = [ctypes.c_int]
        L.wdr_default_solver_params.argtypes = [ctypes.POINTER(SolverParams)]
        L.wdr_default_solver_params.restype = None
        L.wdr_ctx_create.argtypes = [ctypes.POINTER(Geom), ctypes.c_int, ctypes.POINTER(P)]
        L.wdr_ctx_destroy.argtypes = [P]
        L.wdr_ctx_volume.argtypes = [P]
        L.wdr_ctx_volume.restype = ctypes.c_int64
        L.wdr_ctx_nblocks.argtypes = [P]
        L.wdr_ctx_nblocks.restype = ctypes.c_int32
        L.wdr_ctx_set_stencil.argtypes = [P, i32]
        L.wdr_ctx_set_mr_form.argtypes = [P, i32]
        L.wdr_ctx_set_cg_form.argtypes = [P, i32]
        L.wdr_traffic.argtypes = [i32]
        L.wdr_traffic.restype = ctypes.c_int64
        L.wdr_site_maps.argtypes = [P, P, P, P, P, P]
        L.wdr_active_links.argtypes = [P, i32, i32, P, P]
        L.wdr_gauge_create.argtypes = [P, P, ctypes.POINTER(P), P]
        L.wdr_gauge_destroy.argtypes = [P]
        L.wdr_gauge_is_su3.argtypes = [P]
        L.wdr_gauge_is_su3.restype = i32
        L.wdr_gauge_set_clover.argtypes = [P, P, d, d, P]
        L.wdr_clover_field.argtypes = [P, P, i32, P, P]
        L.wdr_interpolate.argtypes = [P, P, P, i32, i32, P, P]
        L.wdr_noise.argtypes = [P, ctypes.c_int, ctypes.c_uint64, i32, i32, i32, P, P]
        L.wdr_field_bytes.argtypes = [P, ctypes.c_int]
        L.wdr_field_bytes.restype = ctypes.c_int64
        L.wdr_halo_bytes.argtypes = [P, ctypes.c_int]
        L.wdr_halo_bytes.restype = ctypes.c_int64
        L.wdr_halo_pack.argtypes = [P, P, ctypes.c_int, P, P, P, P]
        L.wdr_halo_unpack.argtypes = [P, P, d, ctypes.c_int, P, P, i32, i32, P, P]
        L.wdr_pack.argtypes = [P, ctypes.c_int, P, P, P]
        L.wdr_unpack.argtypes = [P, ctypes.c_int, P, P, P]
        L.wdr_apply_D_internal.argtypes = [P, P, d, ctypes.c_int, P, P, P]
        L.wdr_eo16_field_bytes.argtypes = [P]
        L.wdr_eo16_field_bytes.restype = ctypes.c_int64
        L.wdr_pack_eo16.argtypes = [P, i32, P, P, P]
        L.wdr_unpack_eo16.argtypes = [P, i32, P, P, P]
        L.wdr_apply_hop_eo_internal.argtypes = [P, P, d, ctypes.c_int, i32, i32, i32, P, P, P, P]
        for f in ("wdr_apply_D", "wdr_apply_D_noalloc"):
            getattr(L, f).argtypes = [P, P, d, ctypes.c_int, P, P, P]
        for f in ("wdr_apply_Dblock", "wdr_apply_Dhop", "wdr_apply_Dee"):
            getattr(L, f).argtypes = [P, P, d, ctypes.c_int, i32, P, P, P]
        L.wdr_sap.argtypes = [P, P, d, ctypes.POINTER(SolverParams), P, P, P]
        L.wdr_solve.argtypes = [P, P, d, ctypes.POINTER(SolverParams), P, P, ctypes.POINTER(SolveInfo), P]
        L.wdr_block_solve.argtypes = [P, P, d, i32, ctypes.POINTER(SolverParams), P, P, ctypes.POINTER(SolveInfo),
                                      P]
        L.wdr_apply_schur.argtypes = [P, P, d, ctypes.POINTER(SolverParams), P, P, P]
        L.wdr_logdet_ratio.argtypes = [P, P, P, d, ctypes.POINTER(EstParams), P, P, ctypes.POINTER(SolveInfo), P]
        L.wdr_logdet_ratio_batch.argtypes = [i32, ctypes.POINTER(Proposal), ctypes.POINTER(EstParams), P, P,
                                             ctypes.POINTER(SolveInfo), P]
        L.wdr_autotune.argtypes = [P, P, P, d, ctypes.POINTER(EstParams), ctypes.POINTER(d), P]
        L.wdr_block_logdet.argtypes = [P, P, d, i32, P, P]
        L.wdr_block_logdet_ratio.argtypes = [P, P, P, d, i32, P, P]
        L.wdr_block_fields.argtypes = [P, P, P, P]
        L.wdr_heatbath.argtypes = [P, d, P, ctypes.c_uint64, i32, P, P]
        L.wdr_overrelax.argtypes = [P, P, P, P]
        L.wdr_relative_gauge.argtypes = [P, P, P, i32, ctypes.POINTER(d), P]
        L.wdr_filter_step.argtypes = [P, d, d, P, i32, ctypes.POINTER(EstParams), ctypes.c_uint64, P, P,
                                      ctypes.POINTER(FilterInfo), P]
        L.wdr_block_schur_ratio.argtypes = [P, P, P, d, P, ctypes.POINTER(EstParams), P, P,
                                            ctypes.POINTER(SolveInfo), P]
        _lib = L
    return _lib


def _sample_tail(op, nblocks):
    """Trailing sample dimensions: one per block for BLOCKS, blocks then the
    Schur complement for DD."""
    return (nblocks,) if op == OP_BLOCKS else (nblocks + 1,) if op == OP_DD else ()


def _check(status: int, allow=(OK,)):
    if status not in allow:
        raise WdrError(status, lib().wdr_last_error().decode())
    return status


def traffic(reset: bool = False) -> int:
    """Compulsory device-memory bytes of the estimates since the last reset."""
    return int(lib().wdr_traffic(int(reset)))


def default_params(**kw) -> SolverParams:
    p = SolverParams()
    lib().wdr_default_solver_params(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _torch():
    import torch
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _dev(t, shape, dtype_name="complex128"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a GPU torch tensor")
    if str(t.dtype) != "torch." + dtype_name:
        raise TypeError("expected dtype %s, got %s" % (dtype_name, t.dtype))
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError("expected a contiguous tensor of shape %s, got %s" % (tuple(shape), tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class Gauge:
    ctx: "Context"
    handle: ctypes.c_void_p

    @property
    def su3(self) -> bool:
        """Every link is SU(3) to 1e-10 (two-row link paths are used)."""
        return bool(lib().wdr_gauge_is_su3(self.handle))

    def __del__(self):
        if self.handle and _lib is not None:
            _lib.wdr_gauge_destroy(self.handle)
            self.handle = None


class Context:
    """A lattice geometry (L, blocks B, boundary phases bc) on one device."""

    def __init__(self, L, B, bc=(1, 1, 1, 1), device: int = 0):
        g = Geom()
        for mu in range(4):
            g.L[mu], g.B[mu], g.bc[mu] = int(L[mu]), int(B[mu]), int(bc[mu])
        h = ctypes.c_void_p()
        _check(lib().wdr_ctx_create(ctypes.byref(g), device, ctypes.byref(h)))
        self.handle = h
        self.L, self.B, self.bc = tuple(L), tuple(B), tuple(bc)
        self.V = int(lib().wdr_ctx_volume(h))
        self.nblocks = int(lib().wdr_ctx_nblocks(h))
        self.device = device

    def set_stencil(self, choice: int):
        """Stencil kernel for D and D_b (STENCIL_AUTO, STENCIL_DIR, STENCIL_BLK)."""
        _check(lib().wdr_ctx_set_stencil(self.handle, int(choice)))

    def set_mr_form(self, choice: int):
        """Launch form of the FP32 / FP16 block MR of block solves (MR_AUTO,
        MR_ONE_PER_CU, MR_TWO_PER_CU)."""
        _check(lib().wdr_ctx_set_mr_form(self.handle, int(choice)))

    def set_cg_form(self, choice: int):
        """Launch form of the CG steps of the FP64 / FP32 even-odd CGNE
        (CG_LAUNCHES, CG_PERSISTENT)."""
        _check(lib().wdr_ctx_set_cg_form(self.handle, int(choice)))

    def close(self):
        if getattr(self, "handle", None):
            _torch().cuda.synchronize()
            lib().wdr_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- tensors
    def _empty(self, *shape, dtype=None):
        torch = _torch()
        return torch.empty(*shape, dtype=dtype or torch.complex128, device="cuda:%d" % self.device)

    def spinor_like(self):
        return self._empty(self.V, 4, 3)

    # ---- geometry
    def site_maps(self):
        torch = _torch()
        out = [self._empty(self.V, dtype=torch.int32) for _ in range(4)]
        _check(lib().wdr_site_maps(self.handle, *[ctypes.c_void_p(t.data_ptr()) for t in out], _stream()))
        return out

    def active_links(self, lo: int, hi: int):
        torch = _torch()
        m = self._empty(self.V, 4, dtype=torch.uint8)
        _check(lib().wdr_active_links(self.handle, lo, hi, ctypes.c_void_p(m.data_ptr()), _stream()))
        return m

    # ---- gauge fields and path
    def gauge(self, U, csw: float = 0.0, kappa: float = 0.0) -> Gauge:
        """Upload U; with csw != 0 attach the clover term for (csw, kappa)."""
        h = ctypes.c_void_p()
        _check(lib().wdr_gauge_create(self.handle, _dev(U, (self.V, 4, 3, 3)), ctypes.byref(h), _stream()))
        g = Gauge(self, h)
        if csw:
            self.set_clover(g, csw, kappa)
        return g

    def set_clover(self, U: Gauge, csw: float, kappa: float):
        """Attach (csw != 0) or remove (csw = 0) the clover term of U."""
        _check(lib().wdr_gauge_set_clover(self.handle, U.handle, float(csw), float(kappa), _stream()))

    def clover_field(self, U: Gauge, inverse: bool = False):
        """A or A^-1 of U's clover term: [V, 12, 12] complex128 on the device."""
        out = self._empty(self.V, 12, 12)
        _check(lib().wdr_clover_field(self.handle, U.handle, int(bool(inverse)), ctypes.c_void_p(out.data_ptr()),
                                      _stream()))
        return out

    def interpolate(self, U, Up, i: int, N: int):
        out = self._empty(self.V, 4, 3, 3)
        shp = (self.V, 4, 3, 3)
        _check(lib().wdr_interpolate(self.handle, _dev(U, shp), _dev(Up, shp), i, N,
                                     ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    # ---- noise and operators
    def noise(self, kind: int, seed: int, step: int, k: int, black_only: bool = False):
        out = self.spinor_like()
        _check(lib().wdr_noise(self.handle, kind, ctypes.c_uint64(seed), step, k, int(black_only),
                               ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    def _op(self, fn, gauge: Gauge, kappa, psi, prec, *extra):
        out = self.spinor_like()
        _check(getattr(lib(), fn)(self.handle, gauge.handle, kappa, prec, *extra,
                                  _dev(psi, (self.V, 4, 3)), ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    # ---- internal-layout fields (flat byte tensors owned by the caller)
    def internal_field(self, prec=F64):
        torch = _torch()
        n = int(lib().wdr_field_bytes(self.handle, prec))
        return self._empty(n, dtype=torch.uint8)

    def pack(self, psi, prec=F64):
        out = self.internal_field(prec)
        _check(lib().wdr_pack(self.handle, prec, _dev(psi, (self.V, 4, 3)), ctypes.c_void_p(out.data_ptr()),
                              _stream()))
        return out

    def unpack(self, f, prec=F64):
        out = self.spinor_like()
        _check(lib().wdr_unpack(self.handle, prec, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                _stream()))
        return out

    def eo16_field(self, nsys: int = 1):
        """Flat byte tensor for nsys half fields in the FP16 layout of the
        even-odd CG."""
        torch = _torch()
        n = int(lib().wdr_eo16_field_bytes(self.handle))
        if n <= 0:
            raise WdrError(EINVAL, "FP16 half fields need 4^4 blocks in a 2-colourable checkerboard")
        return self._empty(n * nsys, dtype=torch.uint8)

    def pack_eo16(self, psi, parity: int):
        out = self.eo16_field()
        _check(lib().wdr_pack_eo16(self.handle, parity, _dev(psi, (self.V, 4, 3)), ctypes.c_void_p(out.data_ptr()),
                                   _stream()))
        return out

    def unpack_eo16(self, f, parity: int):
        out = self.spinor_like()
        _check(lib().wdr_unpack_eo16(self.handle, parity, ctypes.c_void_p(f.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    def apply_hop_eo_internal(self, gauge, kappa, prec, parity, dag, fin, fdiag, fout, nsys: int = 1):
        """out = diag - kappa H_{parity, 1-parity} in (gamma_5-conjugated for dag) on
        internal fields of nsys systems: one kernel launch."""
        _check(lib().wdr_apply_hop_eo_internal(self.handle, gauge.handle, kappa, prec, parity, dag, nsys,
                                               ctypes.c_void_p(fin.data_ptr()),
                                               None if fdiag is None else ctypes.c_void_p(fdiag.data_ptr()),
                                               ctypes.c_void_p(fout.data_ptr()), _stream()))
        return fout

    # ---- halo of a slab cut along t (the context's t boundary open)
    def halo_field(self, prec=F64):
        """Flat byte tensor for one face buffer of half spinors."""
        torch = _torch()
        n = int(lib().wdr_halo_bytes(self.handle, prec))
        return self._empty(n, dtype=torch.uint8)

    def halo_pack(self, U, fin, send_lo, send_hi, prec=F64):
        """send_lo = (1 - g_t) psi on t = 0, send_hi = (1 + g_t) U_t^+ psi on
        the last t slice; U the canonical FP64 links of the slab."""
        _check(lib().wdr_halo_pack(self.handle, _dev(U, (self.V, 4, 3, 3)), prec, ctypes.c_void_p(fin.data_ptr()),
                                   ctypes.c_void_p(send_lo.data_ptr()), ctypes.c_void_p(send_hi.data_ptr()),
                                   _stream()))

    def halo_unpack(self, U, kappa, recv_lo, recv_hi, sign_lo, sign_hi, fout, prec=F64):
        """fout -= kappa (hops across both t faces) from the neighbours' faces."""
        _check(lib().wdr_halo_unpack(self.handle, _dev(U, (self.V, 4, 3, 3)), kappa, prec,
                                     ctypes.c_void_p(recv_lo.data_ptr()), ctypes.c_void_p(recv_hi.data_ptr()),
                                     int(sign_lo), int(sign_hi), ctypes.c_void_p(fout.data_ptr()), _stream()))
        return fout

    def apply_D_internal(self, gauge, kappa, fin, fout, prec=F64):
        _check(lib().wdr_apply_D_internal(self.handle, gauge.handle, kappa, prec, ctypes.c_void_p(fin.data_ptr()),
                                          ctypes.c_void_p(fout.data_ptr()), _stream()))
        return fout

    def apply_D(self, gauge, kappa, psi, prec=F64):
        return self._op("wdr_apply_D", gauge, kappa, psi, prec)

    def apply_D_noalloc(self, gauge, kappa, psi, out, prec=F64):
        """D psi into the caller's out (complex128 [V, 4, 3]) with the library's
        static staging array: no device allocation in the call."""
        _check(lib().wdr_apply_D_noalloc(self.handle, gauge.handle, kappa, prec, _dev(psi, (self.V, 4, 3)),
                                         _dev(out, (self.V, 4, 3)), _stream()))
        return out

    def apply_Dblock(self, gauge, kappa, psi, colour, prec=F64):
        return self._op("wdr_apply_Dblock", gauge, kappa, psi, prec, colour)

    def apply_Dhop(self, gauge, kappa, psi, from_colour, prec=F64):
        return self._op("wdr_apply_Dhop", gauge, kappa, psi, prec, from_colour)

    def apply_Dee(self, gauge, kappa, psi, blocked=False, prec=F64):
        return self._op("wdr_apply_Dee", gauge, kappa, psi, prec, int(blocked))

    # ---- solvers
    def sap(self, gauge, kappa, psi, params: SolverParams):
        out = self.spinor_like()
        _check(lib().wdr_sap(self.handle, gauge.handle, kappa, ctypes.byref(params), _dev(psi, (self.V, 4, 3)),
                             ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    def solve(self, gauge, kappa, b, params: SolverParams, allow_noconv=False):
        out = self.spinor_like()
        info = SolveInfo()
        st = lib().wdr_solve(self.handle, gauge.handle, kappa, ctypes.byref(params), _dev(b, (self.V, 4, 3)),
                             ctypes.c_void_p(out.data_ptr()), ctypes.byref(info), _stream())
        _check(st, (OK, ENOCONV) if allow_noconv else (OK,))
        return out, info

    def block_solve(self, gauge, kappa, colour, b, params: SolverParams):
        out = self.spinor_like()
        info = SolveInfo()
        _check(lib().wdr_block_solve(self.handle, gauge.handle, kappa, colour, ctypes.byref(params),
                                     _dev(b, (self.V, 4, 3)), ctypes.c_void_p(out.data_ptr()), ctypes.byref(info),
                                     _stream()))
        return out, info

    def schur(self, gauge, kappa, psi, params: SolverParams):
        out = self.spinor_like()
        _check(lib().wdr_apply_schur(self.handle, gauge.handle, kappa, ctypes.byref(params),
                                     _dev(psi, (self.V, 4, 3)), ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    def autotune(self, U: Gauge, Up: Gauge, kappa, op, n_steps, n_noise, noise, seed, params: SolverParams):
        """Tuned copy of params (Schwarz and block-solve depths) for estimates
        of this kind on this context, and the time of the chosen schedule."""
        ep = EstParams()
        ep.op, ep.n_steps, ep.n_noise, ep.noise, ep.seed, ep.sp = op, n_steps, n_noise, noise, seed, params
        secs = ctypes.c_double()
        _check(lib().wdr_autotune(self.handle, U.handle, Up.handle, kappa, ctypes.byref(ep), ctypes.byref(secs),
                                  _stream()))
        return ep.sp, secs.value

    def block_logdet(self, U: Gauge, kappa, max_blocks=0, allow_nan=False):
        """Exact log det(D_b^+ D_b) of every block, by lexicographic block id
        (max_blocks: block matrices per pass, 0 for as many as fit in 8 GiB)."""
        out = np.zeros(self.nblocks, dtype=np.float64)
        _check(lib().wdr_block_logdet(self.handle, U.handle, kappa, max_blocks, out.ctypes.data_as(ctypes.c_void_p),
                                      _stream()), (OK, ENOCONV) if allow_nan else (OK,))
        return out

    def block_logdet_ratio(self, U: Gauge, Up: Gauge, kappa, max_blocks=0):
        """Exact block ratios log det(D_b'^+ D_b') - log det(D_b^+ D_b)."""
        out = np.zeros(self.nblocks, dtype=np.float64)
        _check(lib().wdr_block_logdet_ratio(self.handle, U.handle, Up.handle, kappa, max_blocks,
                                            out.ctypes.data_as(ctypes.c_void_p), _stream()))
        return out

    def heatbath(self, beta, mask, seed, sweep, U):
        """One heat-bath sweep of the links marked in mask (uint8 [V, 4]) of the
        canonical field U (complex128 [V, 4, 3, 3] on the device), in place."""
        _check(lib().wdr_heatbath(self.handle, beta, _dev(mask, (self.V, 4), "uint8"), seed, sweep,
                                  _dev(U, (self.V, 4, 3, 3)), _stream()))
        return U

    def relative_gauge(self, U, Up, sweeps):
        """Relative gauge fixing of Up to U (canonical device fields), Up in
        place; returns F = sum Re tr(U'_mu(x) U_mu(x)^+) / 3."""
        F = ctypes.c_double()
        _check(lib().wdr_relative_gauge(self.handle, _dev(U, (self.V, 4, 3, 3)), _dev(Up, (self.V, 4, 3, 3)), sweeps,
                                        ctypes.byref(F), _stream()))
        return F.value

    def overrelax(self, mask, U):
        """One over-relaxation sweep of the masked links of U, in place."""
        _check(lib().wdr_overrelax(self.handle, _dev(mask, (self.V, 4), "uint8"), _dev(U, (self.V, 4, 3, 3)),
                                   _stream()))
        return U

    def filter_step(self, beta, kappa, mask, n_block_steps, n_steps, n_noise, seed, est_seed, params: SolverParams,
                    U):
        """One step of the hierarchical filter on U (in place); n_steps = 0
        runs the block steps only.  Returns (info, block decisions
        [n_block_steps, nblocks])."""
        ep = None
        if n_steps > 0:
            ep = EstParams()
            ep.op, ep.n_steps, ep.n_noise, ep.noise, ep.seed, ep.sp = OP_SCHUR, n_steps, n_noise, NOISE_GAUSS, \
                est_seed, params
        acc = np.zeros((max(n_block_steps, 1), self.nblocks), dtype=np.uint8)
        info = FilterInfo()
        _check(lib().wdr_filter_step(self.handle, beta, kappa, _dev(mask, (self.V, 4), "uint8"), n_block_steps,
                                     ctypes.byref(ep) if ep is not None else None, seed, _dev(U, (self.V, 4, 3, 3)),
                                     acc.ctypes.data_as(ctypes.c_void_p), ctypes.byref(info), _stream()))
        return info, acc[:n_block_steps].astype(bool)

    def block_fields(self, U: Gauge):
        """Links of every block as a lattice of the block's extents:
        [nblocks, V_b, 4, 3, 3] complex128 on the device."""
        Vb = int(np.prod(self.B))
        out = self._empty(self.nblocks * Vb, 4, 3, 3).reshape(self.nblocks, Vb, 4, 3, 3)
        _check(lib().wdr_block_fields(self.handle, U.handle, ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    def block_schur_ratio(self, U: Gauge, Up: Gauge, kappa, sub: "Context", n_steps, n_noise, noise, seed,
                          params: SolverParams, max_batch: int = 0):
        """Recursive DD: the Schur-complement ratio of every block's Dirichlet
        operator over the sub-blocks of `sub` (lattice = one block, open
        boundaries).  Returns (samples [nblocks, n_steps, n_noise], log Rhat
        [nblocks], info)."""
        ep = EstParams()
        ep.op, ep.n_steps, ep.n_noise, ep.noise, ep.seed, ep.sp = OP_SCHUR, n_steps, n_noise, noise, seed, params
        ep.max_batch = max_batch
        samples = np.zeros((self.nblocks, n_steps, n_noise), dtype=np.float64)
        lrs = np.zeros(self.nblocks, dtype=np.float64)
        info = SolveInfo()
        _check(lib().wdr_block_schur_ratio(self.handle, U.handle, Up.handle, kappa, sub.handle, ctypes.byref(ep),
                                           samples.ctypes.data_as(ctypes.c_void_p),
                                           lrs.ctypes.data_as(ctypes.c_void_p), ctypes.byref(info), _stream()))
        return samples, lrs, info

    def logdet_ratio(self, U: Gauge, Up: Gauge, kappa, op, n_steps, n_noise, noise, seed, params: SolverParams,
                     max_batch: int = 0):
        """Returns (samples [n_steps, n_noise] (x nblocks for BLOCKS, x nblocks + 1
        for DD), log Rhat, info)."""
        ep = EstParams()
        ep.op, ep.n_steps, ep.n_noise, ep.noise, ep.seed, ep.sp = op, n_steps, n_noise, noise, seed, params
        ep.max_batch = max_batch
        shape = (n_steps, n_noise) + _sample_tail(op, self.nblocks)
        samples = np.zeros(shape, dtype=np.float64)
        lr = ctypes.c_double()
        info = SolveInfo()
        _check(lib().wdr_logdet_ratio(self.handle, U.handle, Up.handle, kappa, ctypes.byref(ep),
                                      samples.ctypes.data_as(ctypes.c_void_p), ctypes.byref(lr), ctypes.byref(info),
                                      _stream()))
        return samples, lr.value, info


def logdet_ratio_batch(props, op, n_steps, n_noise, noise, params: SolverParams, max_batch: int = 0):
    """Estimates for a list of proposals (ctx, U, Up, kappa, seed), contexts
    possibly of different lattice sizes, in one batched call.  Returns (list of
    sample arrays [n_steps, n_noise] (x nblocks for BLOCKS), log Rhat array, info)."""
    n = len(props)
    arr = (Proposal * n)()
    sizes = []
    for j, (ctx, U, Up, kappa, seed) in enumerate(props):
        arr[j].ctx, arr[j].U, arr[j].Up, arr[j].kappa, arr[j].seed = ctx.handle, U.handle, Up.handle, kappa, seed
        sizes.append((n_steps, n_noise) + _sample_tail(op, ctx.nblocks))
    ep = EstParams()
    ep.op, ep.n_steps, ep.n_noise, ep.noise, ep.seed, ep.sp = op, n_steps, n_noise, noise, 0, params
    ep.max_batch = max_batch
    flat = np.zeros(sum(int(np.prod(z)) for z in sizes), dtype=np.float64)
    lr = np.zeros(n, dtype=np.float64)
    info = SolveInfo()
    _check(lib().wdr_logdet_ratio_batch(n, arr, ctypes.byref(ep), flat.ctypes.data_as(ctypes.c_void_p),
                                        lr.ctypes.data_as(ctypes.c_void_p), ctypes.byref(info), _stream()))
    out, pos = [], 0
    for z in sizes:
        k = int(np.prod(z))
        out.append(flat[pos:pos + k].reshape(z))
        pos += k
    return out, lr, info
