"""Plain FP64 oracle (test infrastructure only; see the package docstring).

Every function cites the passage of the paper it follows.  Fields use the
canonical layout: spinors ``psi[V, 4, 3]`` and gauge fields ``U[V, 4, 3, 3]``
(complex128), ``site = x0 + L0*(x1 + L1*(x2 + L2*x3))``.

Pins (tests under ``tests/test_oracle_*.py``):
  * operator          free-field plane waves (closed form), U(1) background
                      (closed form), gamma5-hermiticity, gauge covariance,
                      free-field log det (closed form)
  * blocks / hops     D = sum of parts; entries equal the masked dense D;
                      det D = prod_b det D_b * det Dhat (Sec. 3, eq. ddfactor);
                      Dhat psi = psi on black-interior support (Sec. 4)
  * even/odd          det D = det(1 - kappa^2 H_eo H_oe) (dense)
  * solver            residual, dense numpy solve
  * SAP / MR          multiplicative Schwarz closed form with dense block
                      inverses; MR residual monotonic; odd-site equations exact
  * noise             Philox4x64-10 vs numpy.random.Philox and published
                      known-answer vectors; moments
  * path              endpoints, SU(3), geodesic step length, scipy
                      fractional_matrix_power; telescoping of eq. param
  * sample            dense -eta^+(M^+M - 1)eta; E[s] = -tr(M^+M - 1)
  * log ratio         exact dense log R; sum of factor log dets (eq. param)
  * block log dets    per-block slices of the dense D_bb + D_ww; eq. ddfactor
                      with the dense Schur complement; small-kappa plaquette
                      expansion (closed form); gauge invariance; locality;
                      open boundaries = Dirichlet block; eq. ddrec
  * heat-bath         Kennedy-Pendleton a0 moments vs Bessel ratio and
                      quadrature; one-link fixed point vs a reweighted Haar
                      integral; SU(3) kept, unmasked links untouched;
                      strong-coupling plaquette beta/18 + beta^2/216
  * over-relaxation   action unchanged, SU(3) kept, one subgroup an
                      involution
  * relative gauge    F never decreases; block determinants unchanged; a
                      gauge copy of U is driven back to U
  * clover term       constant abelian fluxes in a magnetic and an electric
                      plane (closed forms worked out by hand); zero on the
                      unit field; hermitian, chiral, spin-traceless; gauge
                      covariance; a changed link reaches exactly the 14
                      corners of its plaquettes; D_b = D minus the crossing
                      hops; solves and FULL / BLOCKS / SCHUR samples against
                      dense linear algebra
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wdr_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C part of the oracle with gcc (OpenMP)."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        # OpenMP threads that spin between calls starve numpy's BLAS threads
        os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i = ctypes.c_int
        d = ctypes.c_double
        L.oracle_gamma.argtypes = [i, P]
        L.oracle_site_maps.argtypes = [P, P, P, P, P]
        L.oracle_apply_D.argtypes = [P, P, d, P, P, P, P]
        L.oracle_apply_Dblock.argtypes = [P, P, P, d, P, P, i, P, P]
        L.oracle_apply_Dhop.argtypes = [P, P, P, d, P, i, P, P]
        L.oracle_apply_Dee.argtypes = [P, P, P, d, P, i, P, P]
        L.oracle_mul_g5.argtypes = [ctypes.c_long, P, P]
        L.oracle_cgne.argtypes = [P, P, P, d, P, P, i, i, P, P, P, d, i, P]
        L.oracle_cgne.restype = i
        L.oracle_sap.argtypes = [P, P, P, d, P, P, i, i, P, P]
        L.oracle_philox4x64_10.argtypes = [P, P, P]
        L.oracle_noise.argtypes = [P, i, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _pc(clov):
    """Pointer to a clover term [V, 12, 12] (complex128), or NULL."""
    return None if clov is None else _p(clov)


def _i4(v):
    return np.ascontiguousarray(np.asarray(v, dtype=np.int32))


# ----------------------------------------------------------------------------
# Geometry (Sec. 3: blocks, checkerboard colouring, black blocks first)


@dataclass
class Lattice:
    """Periodic 4-d lattice L[0..3] split into blocks B[0..3] (B divides L).

    bc[mu] = +1 periodic, -1 antiperiodic in direction mu.
    """

    L: tuple
    B: tuple = None
    bc: tuple = (1, 1, 1, 1)
    _cache: dict = field(default_factory=dict, repr=False, compare=False)

    def __post_init__(self):
        self.L = tuple(int(v) for v in self.L)
        self.B = tuple(int(v) for v in (self.B if self.B is not None else self.L))
        self.bc = tuple(int(v) for v in self.bc)
        for l, b in zip(self.L, self.B):
            if b <= 0 or l % b:
                raise ValueError("block extent must divide the lattice extent")

    @property
    def V(self) -> int:
        return int(np.prod(self.L))

    @property
    def NB(self) -> tuple:
        return tuple(l // b for l, b in zip(self.L, self.B))

    @property
    def Vb(self) -> int:
        return int(np.prod(self.B))

    @property
    def nblocks(self) -> int:
        return int(np.prod(self.NB))

    def arrays(self):
        return _i4(self.L), _i4(self.B), _i4(self.bc)

    def coords(self) -> np.ndarray:
        """x[site, mu] for every canonical site."""
        s = np.arange(self.V)
        out = np.empty((self.V, 4), dtype=np.int64)
        for mu in range(4):
            out[:, mu] = s % self.L[mu]
            s = s // self.L[mu]
        return out

    def maps(self):
        """(block id, block colour, site parity) per canonical site, from C."""
        if "maps" not in self._cache:
            L, B, _ = self.arrays()
            bid = np.empty(self.V, np.int32)
            col = np.empty(self.V, np.int32)
            par = np.empty(self.V, np.int32)
            lib().oracle_site_maps(_p(L), _p(B), _p(bid), _p(col), _p(par))
            self._cache["maps"] = (bid, col, par)
        return self._cache["maps"]


def block_order(lat: Lattice) -> np.ndarray:
    """Black-first block ordering (Sec. 3, the block form of eq. domdec):
    all black blocks precede all white blocks, each colour's blocks by
    lexicographic block coordinates.  Within a block (an order the paper
    does not fix; chosen here) even sites precede odd sites, each parity
    lexicographic.  Returns perm with perm[position] = canonical site.
    """
    bid, col, par = lat.maps()
    x = lat.coords()
    local = np.zeros(lat.V, dtype=np.int64)
    for mu in (3, 2, 1, 0):
        local = local * lat.B[mu] + (x[:, mu] % lat.B[mu])
    # rank of each block among blocks of the same colour
    nb = lat.nblocks
    bcol = np.zeros(nb, dtype=np.int64)
    bcol[bid] = col
    slot = np.zeros(nb, dtype=np.int64)
    nblack = int(np.sum(bcol == 0))
    slot[bcol == 0] = np.arange(nblack)
    slot[bcol == 1] = nblack + np.arange(nb - nblack)
    keys = np.lexsort((local, par, slot[bid]))
    return keys


def active_links(lat: Lattice, lo: int = 0, hi: int | None = None) -> np.ndarray:
    """Active-link mask (Sec. 3): inside every block, take the region R of
    sites whose in-block coordinates all lie in [lo, hi]; the active links
    are the links with both ends in R and at most one end on the boundary of
    R.  lo = 0, hi = B-1 is the rule for the whole block (about 10% of the
    links for 4^4 blocks, Sec. 5); lo = 1, hi = 6 in 8^4 blocks is the 6^4
    core of Sec. 6 (8%).  Returns mask[site, mu] for the link x -> x+mu.
    """
    x = lat.coords()
    V = lat.V
    mask = np.zeros((V, 4), dtype=bool)
    for mu in range(4):
        h = (hi if hi is not None else lat.B[mu] - 1)
        ok = np.ones(V, dtype=bool)
        for nu in range(4):
            hn = hi if hi is not None else lat.B[nu] - 1
            r = x[:, nu] % lat.B[nu]
            if nu == mu:
                # both ends x, x+mu inside R: lo <= r and r + 1 <= h
                ok &= (r >= lo) & (r + 1 <= h)
            else:
                # both ends share this coordinate; one end interior needs it
                # strictly inside R
                ok &= (r > lo) & (r < hn)
        mask[:, mu] = ok
    return mask


# ----------------------------------------------------------------------------
# Operator (Sec. 5: plain Wilson-Dirac operator with hopping parameter kappa;
# Sec. 3, eq. domdec: Dirichlet blocks and interaction hops)


def gamma(mu: int) -> np.ndarray:
    out = np.empty(32, dtype=np.float64)
    lib().oracle_gamma(mu, _p(out))
    return out.view(np.complex128).reshape(4, 4)


GAMMA5 = np.diag([1.0, 1.0, -1.0, -1.0]).astype(np.complex128)


def _c(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def g5(psi: np.ndarray) -> np.ndarray:
    out = _c(psi).copy()
    out[:, 2:, :] *= -1
    return out


def apply_D(lat: Lattice, U, kappa: float, psi, clov=None) -> np.ndarray:
    """D psi; with clov (clover_term) the diagonal is 1 + T(x)."""
    U, psi = _c(U), _c(psi)
    clov = None if clov is None else _c(clov)
    out = np.empty_like(psi)
    L, _, bc = lat.arrays()
    lib().oracle_apply_D(_p(L), _p(bc), kappa, _p(U), _pc(clov), _p(psi), _p(out))
    return out


def apply_Dblock(lat: Lattice, U, kappa: float, psi, colour: int, clov=None) -> np.ndarray:
    """D_bb (colour 0), D_ww (colour 1) or both (2): Dirichlet block operators
    (their diagonal is that of D, with the clover term when clov is given)."""
    U, psi = _c(U), _c(psi)
    clov = None if clov is None else _c(clov)
    out = np.empty_like(psi)
    L, B, bc = lat.arrays()
    lib().oracle_apply_Dblock(_p(L), _p(B), _p(bc), kappa, _p(U), _pc(clov), colour, _p(psi), _p(out))
    return out


def apply_Dhop(lat: Lattice, U, kappa: float, psi, from_colour: int) -> np.ndarray:
    """Block-interaction hops: from_colour 1 gives D_bw, 0 gives D_wb."""
    U, psi = _c(U), _c(psi)
    out = np.empty_like(psi)
    L, B, bc = lat.arrays()
    lib().oracle_apply_Dhop(_p(L), _p(B), _p(bc), kappa, _p(U), from_colour, _p(psi), _p(out))
    return out


def apply_Dee(lat: Lattice, U, kappa: float, psi, blocked: bool = False) -> np.ndarray:
    """(1 - kappa^2 H_eo H_oe) psi_e, global or with in-block hops only."""
    U, psi = _c(U), _c(psi)
    out = np.empty_like(psi)
    L, B, bc = lat.arrays()
    lib().oracle_apply_Dee(_p(L), _p(B), _p(bc), kappa, _p(U), int(blocked), _p(psi), _p(out))
    return out


# ----------------------------------------------------------------------------
# Clover term (Sheikholeslami-Wohlert).  Sec. 3 defines the active links for
# Wilson fermions with clover term and Sec. 7 names the clover action as the
# next one; the paper does not write the term out, so this is the standard
# one (Sheikholeslami and Wohlert, Nucl. Phys. B 259 (1985) 572; Luscher,
# Sint, Sommer and Weisz, Nucl. Phys. B 478 (1996) 365), in the hopping
# normalisation of D = 1 - kappa H used here:
#     D = 1 + T - kappa H,   T(x) = c_sw kappa (i/2) sum_{mu,nu} sigma_{mu nu} Fhat_{mu nu}(x),
#     sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu],
#     Fhat_{mu nu}(x) = (Q_{mu nu}(x) - Q_{nu mu}(x)) / 8,
# Q_{mu nu}(x) the sum of the four plaquettes of the (mu, nu) plane that
# begin and end at x, each run mu-side first.  The gauge loops are closed, so
# the fermion boundary phases do not enter.


def sigma(mu: int, nu: int) -> np.ndarray:
    """sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu] (4 x 4)."""
    a, b = gamma(mu), gamma(nu)
    return 0.5j * (a @ b - b @ a)


def _nbr(lat: Lattice, mu: int, d: int) -> np.ndarray:
    """Canonical index of x + d mu-hat for every site x (periodic)."""
    x = lat.coords()
    x[:, mu] = (x[:, mu] + d) % lat.L[mu]
    return x[:, 0] + lat.L[0] * (x[:, 1] + lat.L[1] * (x[:, 2] + lat.L[2] * x[:, 3]))


def clover_leaves(lat: Lattice, U, mu: int, nu: int) -> np.ndarray:
    """Q_{mu nu}(x) [V, 3, 3]: the four plaquettes of the (mu, nu) plane at x,
    each a closed path from x, taken in the same sense of rotation."""
    U = _c(U)
    dag = lambda m: np.conj(np.swapaxes(m, -1, -2))
    Um, Un = U[:, mu], U[:, nu]
    fm, bm, fn, bn = _nbr(lat, mu, 1), _nbr(lat, mu, -1), _nbr(lat, nu, 1), _nbr(lat, nu, -1)
    bm_fn = fn[bm]  # x - mu + nu
    bm_bn = bn[bm]  # x - mu - nu
    fm_bn = bn[fm]  # x + mu - nu
    # x -> x+mu -> x+mu+nu -> x+nu -> x
    Q = Um @ Un[fm] @ dag(Um[fn]) @ dag(Un)
    # x -> x+nu -> x-mu+nu -> x-mu -> x
    Q = Q + Un @ dag(Um[bm_fn]) @ dag(Un[bm]) @ Um[bm]
    # x -> x-mu -> x-mu-nu -> x-nu -> x
    Q = Q + dag(Um[bm]) @ dag(Un[bm_bn]) @ Um[bm_bn] @ Un[bn]
    # x -> x-nu -> x+mu-nu -> x+mu -> x
    Q = Q + dag(Un[bn]) @ Um[bn] @ Un[fm_bn] @ dag(Um)
    return Q


def field_strength(lat: Lattice, U, mu: int, nu: int) -> np.ndarray:
    """Fhat_{mu nu}(x) = (Q_{mu nu} - Q_{nu mu}) / 8 [V, 3, 3]."""
    return (clover_leaves(lat, U, mu, nu) - clover_leaves(lat, U, nu, mu)) / 8.0


def clover_term(lat: Lattice, U, csw: float, kappa: float) -> np.ndarray:
    """T(x) = c_sw kappa (i/2) sum_{mu != nu} sigma_{mu nu} (x) Fhat_{mu nu}(x)
    as [V, 12, 12], row and column index 3 * spin + colour (the layout of
    psi[V, 4, 3] flattened), so that (1 + T(x)) psi(x) is the diagonal term
    of D."""
    T = np.zeros((lat.V, 4, 3, 4, 3), dtype=np.complex128)
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            F = field_strength(lat, U, mu, nu)
            T += np.einsum("st,xab->xsatb", sigma(mu, nu), F)
    return (csw * kappa * 0.5j) * T.reshape(lat.V, 12, 12)


def colour_mask(lat: Lattice, colour: int) -> np.ndarray:
    _, col, _ = lat.maps()
    return col == colour


# ----------------------------------------------------------------------------
# Solvers ("one inversion for each factor", Sec. 4)


class NoConvergence(RuntimeError):
    pass


def solve(lat: Lattice, U, kappa: float, b, op: str = "full", colour: int = 2, tol: float = 1e-13,
          maxit: int = 100000, clov=None):
    """Solve A x = b, A = D (op 'full') or the Dirichlet blocks of one colour
    (op 'block'), with the clover term clov when given, by CG on A A^+ y = b.
    Returns (x, y, iterations, true relative residual)."""
    U, b = _c(U), _c(b)
    clov = None if clov is None else _c(clov)
    x = np.empty_like(b)
    y = np.empty_like(b)
    res = ctypes.c_double()
    L, B, bc = lat.arrays()
    it = lib().oracle_cgne(_p(L), _p(B), _p(bc), kappa, _p(U), _pc(clov), 0 if op == "full" else 1, colour, _p(b),
                           _p(x), _p(y), tol, maxit, ctypes.byref(res))
    if it < 0:
        raise NoConvergence("oracle CGNE did not reach %g (residual %g)" % (tol, res.value))
    return x, y, it, res.value


def sap(lat: Lattice, U, kappa: float, eta, ncy: int, nmr: int, clov=None) -> np.ndarray:
    """Schwarz alternating procedure with ncy cycles and nmr even-odd MR
    steps per block (Luscher hep-lat/0310048, cited in Secs. 1 and 3); with
    clov (clover_term) the block systems carry the clover diagonal."""
    U, eta = _c(U), _c(eta)
    clov = None if clov is None else _c(clov)
    x = np.empty_like(eta)
    L, B, bc = lat.arrays()
    lib().oracle_sap(_p(L), _p(B), _p(bc), kappa, _p(U), _pc(clov), ncy, nmr, _p(eta), _p(x))
    return x


def schur_apply(lat: Lattice, U, kappa: float, eta, block_tol: float = 1e-14, clov=None) -> np.ndarray:
    """Dhat eta = eta - D_bb^-1 D_bw D_ww^-1 D_wb eta on black sites
    (Sec. 3, eq. ddfactor).  White sites of the result are zero."""
    black = colour_mask(lat, 0)
    e = _c(eta).copy()
    e[~black] = 0
    t = apply_Dhop(lat, U, kappa, e, from_colour=0)                        # D_wb eta   (white)
    t, _, _, _ = solve(lat, U, kappa, t, "block", 1, block_tol, clov=clov)  # D_ww^-1   (white)
    t = apply_Dhop(lat, U, kappa, t, from_colour=1)                        # D_bw ...   (black)
    t, _, _, _ = solve(lat, U, kappa, t, "block", 0, block_tol, clov=clov)  # D_bb^-1   (black)
    out = e - t
    out[~black] = 0
    return out


# ----------------------------------------------------------------------------
# Noise (Sec. 4: complex Gaussian noise, fresh for every factor)


def philox4x64_10(counter, key) -> np.ndarray:
    c = np.asarray(counter, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.empty(4, dtype=np.uint64)
    lib().oracle_philox4x64_10(_p(c), _p(k), _p(out))
    return out


NOISE_Z2, NOISE_GAUSS = 0, 1


def noise(lat: Lattice, kind: int, seed: int, step: int, k: int, support=None) -> np.ndarray:
    """Noise vector for path step `step`, sample k; support is None (all
    sites) or a boolean site mask."""
    out = np.empty((lat.V, 4, 3), dtype=np.complex128)
    L = _i4(lat.L)
    m = None if support is None else np.ascontiguousarray(support, dtype=np.uint8)
    lib().oracle_noise(_p(L), kind, ctypes.c_uint64(seed), step, k, None if m is None else _p(m), _p(out))
    return out


# ----------------------------------------------------------------------------
# Path U_0 = U, ..., U_N = U' (Sec. 4, eq. param)


def interpolate(U, Up, i: int, N: int) -> np.ndarray:
    """U_i = exp((i/N) log W) U with W = U' U^+ per link (the geodesic from U
    to U'; the paper only asks ||U_i - U_{i+1}|| ~ 1/N).  log W is taken from
    the eigen-decomposition of W with principal angles in (-pi, pi]; if they
    sum to +-2 pi, the largest (smallest) angle is moved by -+2 pi so that
    log W is traceless and U_i stays in SU(3).  U_0 = U and U_N = U'
    exactly; links with U' == U are copied."""
    U = _c(U)
    Up = _c(Up)
    if i == 0:
        return U.copy()
    if i == N:
        return Up.copy()
    t = i / N
    out = U.copy()
    same = np.all((U == Up).reshape(U.shape[0], 4, 9), axis=2)
    idx = np.nonzero(~same)
    if len(idx[0]) == 0:
        return out
    u = U[idx]
    W = Up[idx] @ np.conj(np.swapaxes(u, -1, -2))
    lam, vec = np.linalg.eig(W)
    th = np.angle(lam)
    s = th.sum(axis=1)
    j_hi = np.argmax(th, axis=1)
    j_lo = np.argmin(th, axis=1)
    r = np.arange(len(th))
    fix_hi = s > np.pi
    fix_lo = s < -np.pi
    th[r[fix_hi], j_hi[fix_hi]] -= 2 * np.pi
    th[r[fix_lo], j_lo[fix_lo]] += 2 * np.pi
    ph = np.exp(1j * t * th)
    Wt = vec @ (ph[:, :, None] * np.linalg.inv(vec))
    out[idx] = Wt @ u
    return out


# ----------------------------------------------------------------------------
# Stochastic estimator (Sec. 4)

OP_FULL, OP_SCHUR, OP_BLOCKS = 0, 1, 2


def _dot(a, b) -> complex:
    return complex(np.vdot(a.ravel(), b.ravel()))


def sample(lat: Lattice, U0, U1, kappa: float, op: int, eta, tol: float = 1e-13, block_tol: float = 1e-14,
           csw: float = 0.0):
    """One sample s = -eta^+ (M^+ M - 1) eta, M = X'^-1 X with X = D (FULL),
    X = the Dirichlet blocks (BLOCKS, one value per block) or X = Dhat
    (SCHUR), X built on U0 and X' on U1 (Sec. 4); csw != 0 adds the clover
    term with that coefficient to D (and so to its blocks and Dhat).

    E over complex Gaussian eta of exp(s) is det(M^+ M)^-1 =
    det(X'^+ X') / det(X^+ X), the ratio the acceptance step needs.

    ||M eta||^2 = ||P z||^2 with z = A'^-1 y is evaluated as
    ||P z~||^2 + 2 Re w^+ (y - A' z~), A'^+ w = P z~, which equals it up to
    ||A'^-1 (y - A' z~)||^2 (both solves tight).

    s itself is the sum over sites of |eta(x)|^2 - |P z(x)|^2 - 2 Re w(x)^+
    r(x), the difference taken per site in FP64 and the sum correctly
    rounded (math.fsum): s is a small difference of two sums of order 12 V,
    whose separate rounding would cost up to ~1e-8 absolute at 32^4.
    """
    eta = _c(eta)
    c0 = clover_term(lat, U0, csw, kappa) if csw else None
    c1 = clover_term(lat, U1, csw, kappa) if csw else None
    if op == OP_FULL:
        y = apply_D(lat, U0, kappa, eta, c0)
        z, w, _, _ = solve(lat, U1, kappa, y, "full", 2, tol, clov=c1)
        # with CGNE, z = A'^+ w exactly, so w solves A'^+ w = z
        r = y - apply_D(lat, U1, kappa, z, c1)
        return math.fsum(_site_terms(eta, z, w, r))
    if op == OP_BLOCKS:
        bid, _, _ = lat.maps()
        y = apply_Dblock(lat, U0, kappa, eta, 2, c0)
        z, w, _, _ = solve(lat, U1, kappa, y, "block", 2, block_tol, clov=c1)
        r = y - apply_Dblock(lat, U1, kappa, z, 2, c1)
        per_site = _site_terms(eta, z, w, r)
        return np.array([math.fsum(per_site[bid == b]) for b in range(lat.nblocks)])
    if op == OP_SCHUR:
        black = colour_mask(lat, 0)
        e = eta.copy()
        e[~black] = 0
        phi = schur_apply(lat, U0, kappa, e, block_tol, clov=c0)
        y = apply_Dblock(lat, U1, kappa, phi, 0, c1)                     # A' Dhat eta, black
        z, _, _, _ = solve(lat, U1, kappa, y, "full", 2, tol, clov=c1)   # D' z = [y; 0]
        pz = z.copy()
        pz[~black] = 0
        # adjoint: D'^+ w = P z  <=>  D' (g5 w) = g5 P z
        v, _, _, _ = solve(lat, U1, kappa, g5(pz), "full", 2, tol, clov=c1)
        w = g5(v)
        r = y - apply_D(lat, U1, kappa, z, c1)
        return math.fsum(_site_terms(e, pz, w, r))
    raise ValueError("unknown operator")


def _site_terms(eta, z, w, r) -> np.ndarray:
    """|eta(x)|^2 - |z(x)|^2 - 2 Re w(x)^+ r(x) per site (Sec. 4 sample,
    second-order form)."""
    return ((np.abs(eta) ** 2).sum(axis=(1, 2)) - (np.abs(z) ** 2).sum(axis=(1, 2))
            - 2 * np.real(np.conj(w) * r).sum(axis=(1, 2)))


def noise_support(lat: Lattice, op: int):
    return colour_mask(lat, 0) if op == OP_SCHUR else None


def log_mean_exp(s: np.ndarray, axis: int = 0) -> np.ndarray:
    m = np.max(s, axis=axis, keepdims=True)
    return np.squeeze(m, axis=axis) + np.log(np.mean(np.exp(s - m), axis=axis))


def combine(samples: np.ndarray) -> np.ndarray:
    """log Rhat = sum_i log( (1/K) sum_k exp(s_{i,k}) ) over the factors of
    eq. param; samples[i, k] (or samples[i, k, block])."""
    return np.sum(log_mean_exp(samples, axis=1), axis=0)


def logdet_ratio(lat: Lattice, U, Up, kappa: float, op: int, n_steps: int, n_noise: int, kind: int, seed: int,
                 tol: float = 1e-13, block_tol: float = 1e-14, csw: float = 0.0):
    """Stochastic estimate of log det(X'^+ X') / det(X^+ X) along the path
    U_0 = U ... U_N = U' (eq. param), one noise vector per factor and sample;
    csw != 0: with the clover term.  Returns (samples, log Rhat)."""
    support = noise_support(lat, op)
    shape = (n_steps, n_noise) + ((lat.nblocks,) if op == OP_BLOCKS else ())
    samples = np.zeros(shape)
    Ui = interpolate(U, Up, 0, n_steps)
    for i in range(n_steps):
        Ui1 = interpolate(U, Up, i + 1, n_steps)
        for k in range(n_noise):
            eta = noise(lat, kind, seed, i, k, support)
            samples[i, k] = sample(lat, Ui, Ui1, kappa, op, eta, tol, block_tol, csw)
        Ui = Ui1
    return samples, combine(samples)


# ----------------------------------------------------------------------------
# Dense forms (small lattices only)


def dense(apply, n_sites: int, cols=None) -> np.ndarray:
    """Dense matrix of a linear map on canonical spinor fields, column by
    column (cols: subset of the 12*V unit vectors)."""
    n = 12 * n_sites
    cols = np.arange(n) if cols is None else np.asarray(cols)
    M = np.empty((n, len(cols)), dtype=np.complex128)
    e = np.zeros((n_sites, 4, 3), dtype=np.complex128)
    flat = e.reshape(-1)
    for j, c in enumerate(cols):
        flat[c] = 1.0
        M[:, j] = apply(e).reshape(-1)
        flat[c] = 0.0
    return M


def log_abs_det(M: np.ndarray) -> float:
    sign, ld = np.linalg.slogdet(M)
    return float(ld)


def exact_log_ratio(lat: Lattice, U, Up, kappa: float, csw: float = 0.0) -> float:
    """log det(D'^+ D') - log det(D^+ D) = 2 (log|det D'| - log|det D|) by
    dense LU (Sec. 2, two-step acceptance); csw != 0: with the clover term."""
    c0 = clover_term(lat, U, csw, kappa) if csw else None
    c1 = clover_term(lat, Up, csw, kappa) if csw else None
    D0 = dense(lambda v: apply_D(lat, U, kappa, v, c0), lat.V)
    D1 = dense(lambda v: apply_D(lat, Up, kappa, v, c1), lat.V)
    return 2.0 * (log_abs_det(D1) - log_abs_det(D0))


def block_log_dets(lat: Lattice, U, kappa: float, blocks=None, clov=None) -> np.ndarray:
    """log det(D_b^+ D_b) = 2 log|det D_b| of the Dirichlet operator of every
    block b (Sec. 3, eq. ddfactor: the block factors; eq. 4step: their ratios
    decide the first acceptance step), by dense LU of the 12 Vb x 12 Vb block
    matrix; with clov (clover_term) the blocks carry the clover diagonal.
    Indexed by lexicographic block id; `blocks` restricts the work to a
    subset (the other entries are NaN).

    Dirichlet blocks do not couple, so a unit vector placed at the same
    in-block position of every block gives that column of every block
    matrix in one application of D_bb + D_ww."""
    bid, _, _ = lat.maps()
    nb, Vb = lat.nblocks, lat.Vb
    blocks = np.arange(nb) if blocks is None else np.asarray(blocks)
    # sites of block b in canonical order, i.e. lexicographic in-block order
    sites = np.argsort(bid, kind="stable").reshape(nb, Vb)
    n = 12 * Vb
    mats = np.empty((len(blocks), n, n), dtype=np.complex128)
    e = np.zeros((lat.V, 12), dtype=np.complex128)
    for loc in range(Vb):
        for c in range(12):
            e[sites[:, loc], c] = 1.0
            out = apply_Dblock(lat, U, kappa, e.reshape(lat.V, 4, 3), 2, clov).reshape(lat.V, 12)
            e[sites[:, loc], c] = 0.0
            for i, b in enumerate(blocks):
                mats[i, :, 12 * loc + c] = out[sites[b]].reshape(-1)
    res = np.full(nb, np.nan)
    for i, b in enumerate(blocks):
        res[b] = 2.0 * log_abs_det(mats[i])
    return res


def site_dofs(mask: np.ndarray) -> np.ndarray:
    """Indices of the 12 components of every site where mask is true."""
    s = np.nonzero(mask)[0]
    return (12 * s[:, None] + np.arange(12)[None, :]).ravel()


# ----------------------------------------------------------------------------
# Gauge update and hierarchical filter (Sec. 2 hierarchical acceptance steps;
# Sec. 3 eq. 4step; Sec. 5: heat-bath of the active links with the Wilson
# plaquette action, block acceptance with the exact block determinants,
# global acceptance with the stochastic Schur-complement estimate)

HB_TAG, ACC_TAG, HB_TRIALS = 5, 6, 64
SUBGROUPS = ((0, 1), (0, 2), (1, 2))


def uniforms(words) -> np.ndarray:
    """53-bit uniforms in (0, 1) from Philox words (as for the noise)."""
    w = np.asarray(words, dtype=np.uint64) >> np.uint64(11)
    return (w.astype(np.float64) + 0.5) * 2.0 ** -53


def kp_a0(alpha, u):
    """One trial of Kennedy and Pendleton (Phys. Lett. B 156 (1985) 393) for
    a0 with density sqrt(1 - a0^2) exp(alpha a0) on [-1, 1], from four
    uniforms u[0..3] (arrays allowed): returns (accepted, a0)."""
    x = -(np.log(u[0]) + np.cos(2.0 * np.pi * u[1]) ** 2 * np.log(u[2])) / alpha
    return u[3] * u[3] <= 1.0 - 0.5 * x, 1.0 - x


def _shift(lat: Lattice, s, mu, d):
    """Canonical index of the periodic neighbour x + d mu-hat (the gauge action
    is periodic whatever the fermion boundary phases)."""
    x = lat.coords()[s].copy()
    x[mu] = (x[mu] + d) % lat.L[mu]
    return int(x[0] + lat.L[0] * (x[1] + lat.L[1] * (x[2] + lat.L[2] * x[3])))


def staple(lat: Lattice, U, s, mu) -> np.ndarray:
    """A with Re tr(U_mu(x) A) the sum of the six plaquettes through the link."""
    dag = lambda m: m.conj().T
    A = np.zeros((3, 3), dtype=np.complex128)
    xm = _shift(lat, s, mu, 1)
    for nu in range(4):
        if nu == mu:
            continue
        xn = _shift(lat, s, nu, 1)
        xd = _shift(lat, s, nu, -1)
        xmd = _shift(lat, xm, nu, -1)
        A += U[xm, nu] @ dag(U[xn, mu]) @ dag(U[s, nu])
        A += dag(U[xmd, nu]) @ dag(U[xd, mu]) @ U[xd, nu]
    return A


def heatbath_link(u, A, beta: float, seed: int, site: int, mu: int, sweep: int) -> np.ndarray:
    """Cabibbo-Marinari heat-bath update (Phys. Lett. B 119 (1982) 387) of
    one link u with staple sum A for the Wilson plaquette action (Sec. 5):
    the SU(2) subgroups (0,1), (0,2), (1,2) in turn.  Subgroup g: W = u A
    restricted to the subgroup is k v with v in SU(2); Y with density
    exp(2 beta k y0 / 3) (Kennedy-Pendleton a0, isotropic direction) gives
    X = Y v^+ and u <- X u.  Random numbers: Philox4x64-10, key (seed, 5),
    counter (site, sweep 2^32 + mu 2^8 + g, trial, j): j = 0 the four
    uniforms of a Kennedy-Pendleton trial, j = 1 cos(theta) = 2 u - 1 and
    phi = 2 pi u' of the accepted trial.  A subgroup that rejects HB_TRIALS
    trials stays unchanged."""
    u = np.array(u, dtype=np.complex128, copy=True)
    for g, (i, j) in enumerate(SUBGROUPS):
        W = u @ A
        a = 0.5 * (W[i, i] + np.conj(W[j, j]))
        b = 0.5 * (W[i, j] - np.conj(W[j, i]))
        k = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
        alpha = 2.0 * beta * k / 3.0
        ctr1 = (int(sweep) << 32) | (mu << 8) | g
        a0 = None
        for t in range(HB_TRIALS):
            ok, x0 = kp_a0(alpha, uniforms(philox4x64_10((site, ctr1, t, 0), (seed, HB_TAG))))
            if ok:
                a0 = x0
                break
        if a0 is None:
            continue
        w = uniforms(philox4x64_10((site, ctr1, t, 1), (seed, HB_TAG)))
        c, phi = 2.0 * w[0] - 1.0, 2.0 * np.pi * w[1]
        r = np.sqrt(max(0.0, 1.0 - a0 * a0))
        sn = np.sqrt(max(0.0, 1.0 - c * c))
        y1, y2, y3 = r * sn * np.cos(phi), r * sn * np.sin(phi), r * c
        Y = np.array([[a0 + 1j * y3, y2 + 1j * y1], [-y2 + 1j * y1, a0 - 1j * y3]])
        v = np.array([[a, b], [-np.conj(b), np.conj(a)]]) / k
        E = np.eye(3, dtype=np.complex128)
        E[np.ix_((i, j), (i, j))] = Y @ v.conj().T
        u = E @ u
    return u


def heatbath(lat: Lattice, U, beta: float, mask, seed: int, sweep: int) -> np.ndarray:
    """One heat-bath sweep of the links where mask[site, mu] is true
    (heatbath_link): mu = 0..3, within each the sites of even then odd
    parity; links of one such class share no plaquette, so their order does
    not matter."""
    U = np.array(U, dtype=np.complex128, copy=True)
    par = lat.coords().sum(axis=1) & 1
    for mu in range(4):
        for p in (0, 1):
            for s in np.nonzero(np.asarray(mask)[:, mu] & (par == p))[0]:
                U[s, mu] = heatbath_link(U[s, mu], staple(lat, U, s, mu), beta, seed, int(s), mu, sweep)
    return U


def overrelax_link(u, A) -> np.ndarray:
    """Over-relaxation of one link u with staple sum A (Sec. 5 names it beside
    the heat-bath): for each SU(2) subgroup (0,1), (0,2), (1,2) in turn, with
    the subgroup part of W = u A equal to k v (v in SU(2)), u <- X u with
    X = (v^+)^2, the reflection through the maximum v^+ of Re tr(X W); it
    leaves Re tr(X W), and hence the action, unchanged."""
    u = np.array(u, dtype=np.complex128, copy=True)
    for i, j in SUBGROUPS:
        W = u @ A
        a = 0.5 * (W[i, i] + np.conj(W[j, j]))
        b = 0.5 * (W[i, j] - np.conj(W[j, i]))
        k = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
        if not k > 0:
            continue
        vd = (np.array([[a, b], [-np.conj(b), np.conj(a)]]) / k).conj().T
        E = np.eye(3, dtype=np.complex128)
        E[np.ix_((i, j), (i, j))] = vd @ vd
        u = E @ u
    return u


def overrelax(lat: Lattice, U, mask) -> np.ndarray:
    """One over-relaxation sweep of the masked links, in the order of
    heatbath."""
    U = np.array(U, dtype=np.complex128, copy=True)
    par = lat.coords().sum(axis=1) & 1
    for mu in range(4):
        for p in (0, 1):
            for s in np.nonzero(np.asarray(mask)[:, mu] & (par == p))[0]:
                U[s, mu] = overrelax_link(U[s, mu], staple(lat, U, s, mu))
    return U


def relative_gauge_functional(U, Up) -> float:
    """F = sum_{x,mu} Re tr(U'_mu(x) U_mu(x)^+) / 3, at most 4 V."""
    return float(np.einsum("xmab,xmab->", Up, U.conj()).real / 3.0)


def relative_gauge(lat: Lattice, U, Up, sweeps: int) -> np.ndarray:
    """Relative gauge fixing of U' to U (Sec. 4: it reduces the spread of the
    eigenvalues of M^+ M): local maximisation of F over gauge transformations
    U'_mu(x) -> g(x) U'_mu(x) g(x+mu)^+, which leave every determinant
    unchanged.  A sweep visits the even, then the odd sites (sites of one
    parity share no link); at site x, with
    K = sum_mu [U'_mu(x) U_mu(x)^+ + U'_mu(x-mu)^+ U_mu(x-mu)],
    h is built from the identity by the subgroups (0,1), (0,2), (1,2): with
    the subgroup part of h K equal to k v, h <- v^+ h (the maximum of
    Re tr(X h K) in the subgroup); then U'_mu(x) <- h U'_mu(x) and
    U'_mu(x-mu) <- U'_mu(x-mu) h^+.  Periodic in every direction."""
    Up = np.array(Up, dtype=np.complex128, copy=True)
    par = lat.coords().sum(axis=1) & 1
    dag = lambda m: m.conj().T
    for _ in range(sweeps):
        for p in (0, 1):
            for s in np.nonzero(par == p)[0]:
                K = np.zeros((3, 3), dtype=np.complex128)
                back = [_shift(lat, s, mu, -1) for mu in range(4)]
                for mu in range(4):
                    K += Up[s, mu] @ dag(U[s, mu]) + dag(Up[back[mu], mu]) @ U[back[mu], mu]
                h = np.eye(3, dtype=np.complex128)
                for i, j in SUBGROUPS:
                    W = h @ K
                    a = 0.5 * (W[i, i] + np.conj(W[j, j]))
                    b = 0.5 * (W[i, j] - np.conj(W[j, i]))
                    k = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
                    if not k > 0:
                        continue
                    E = np.eye(3, dtype=np.complex128)
                    E[np.ix_((i, j), (i, j))] = dag(np.array([[a, b], [-np.conj(b), np.conj(a)]]) / k)
                    h = E @ h
                for mu in range(4):
                    Up[s, mu] = h @ Up[s, mu]
                    Up[back[mu], mu] = Up[back[mu], mu] @ dag(h)
    return Up


def plaquette(lat: Lattice, U) -> float:
    """Mean of Re tr U_P / 3 over all plaquettes (periodic)."""
    tot = 0.0
    for s in range(lat.V):
        for mu in range(4):
            xm = _shift(lat, s, mu, 1)
            for nu in range(mu + 1, 4):
                xn = _shift(lat, s, nu, 1)
                P = U[s, mu] @ U[xm, nu] @ U[xn, mu].conj().T @ U[s, nu].conj().T
                tot += np.trace(P).real / 3.0
    return tot / (6 * lat.V)


def accept(r: float, u: float) -> bool:
    """Metropolis decision with probability min(1, exp(r)) (Sec. 2)."""
    return bool(r >= 0.0 or u < np.exp(r))


def filter_step(lat: Lattice, U, beta: float, kappa: float, mask, n_block_steps: int, n_steps: int, n_noise: int,
                seed: int, est_seed: int):
    """eq. 4step with one level: the three-step algorithm of Sec. 5.
    n_block_steps times: a heat-bath sweep of the masked links (step 0),
    then every block accepted with probability min(1, det(D_b'^+ D_b') /
    det(D_b^+ D_b)) from the exact block determinants (step 1, uniform from
    Philox key (seed, 6), counter (block, step, 0, 0)).  Then the result U'
    is accepted with probability min(1, exp(log Rhat)), log Rhat the
    stochastic estimate of the Schur-complement ratio from U to U' (Sec. 4:
    n_steps factors x n_noise Gaussian noise vectors, key est_seed; uniform
    from counter (0, 0, 1, 0)).  The mask must hold links with both ends in
    one block.  n_steps = 0 runs the block steps only and keeps their
    result.  Returns (field, block accepts [n_block_steps, nblocks], log Rhat,
    global accept)."""
    bid, _, _ = lat.maps()
    cur = np.array(U, dtype=np.complex128, copy=True)
    acc = np.zeros((n_block_steps, lat.nblocks), dtype=bool)
    for st in range(n_block_steps):
        prop = heatbath(lat, cur, beta, mask, seed, st)
        r = block_log_dets(lat, prop, kappa) - block_log_dets(lat, cur, kappa)
        for b in range(lat.nblocks):
            acc[st, b] = accept(r[b], uniforms(philox4x64_10((b, st, 0, 0), (seed, ACC_TAG)))[0])
        take = acc[st][bid]
        cur = np.where(take[:, None, None, None], prop, cur)
    if n_steps == 0:
        return cur, acc, 0.0, True
    _, lr = logdet_ratio(lat, U, cur, kappa, OP_SCHUR, n_steps, n_noise, NOISE_GAUSS, est_seed)
    log_r = float(np.sum(lr))
    ok = accept(log_r, uniforms(philox4x64_10((0, 0, 1, 0), (seed, ACC_TAG)))[0])
    return (cur if ok else np.array(U, dtype=np.complex128, copy=True)), acc, log_r, ok
