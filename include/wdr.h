/*
 * wdr.h -- C ABI of the MI355X library for stochastic estimates of Wilson
 * fermion-determinant ratios det(D'^+ D') / det(D^+ D) (Leder, Finkenrath,
 * Knechtli, "Fermions as global correction in lattice QCD", Lattice 2011).
 *
 * Conventions shared by every call
 * --------------------------------
 * Lattice: extents L[0..3], site = x0 + L0*(x1 + L1*(x2 + L2*x3)); mu = 3 is
 * "time".  Blocks (paper Sec. 3): extents B[0..3] dividing L, every B[mu]
 * even; block colour = (sum_mu floor(x_mu / B_mu)) mod 2, black = 0.  Calls
 * that use the block decomposition need L[mu]/B[mu] even in every direction
 * (a 2-colourable checkerboard); otherwise they return WDR_EINVAL.
 *
 * Canonical fields (what callers pass): FP64 complex, interleaved re/im.
 *   spinor  [site][spin 4][colour 3][2]        12 complex per site
 *   gauge   [site][mu 4][row 3][col 3][2]      U_mu(x), the link x -> x+mu
 * Operator (paper Sec. 5, "plain Wilson-Dirac operator"):
 *   (D psi)(x) = psi(x) - kappa sum_mu [(1 - g_mu) U_mu(x) psi(x+mu)
 *                                      + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu)]
 * chiral basis, g_k = [[0, -i s_k], [i s_k, 0]] (mu = 0,1,2 -> k = 1,2,3),
 * g_4 = [[0, 1], [1, 0]] (mu = 3), g_5 = diag(1, 1, -1, -1); a hop that wraps
 * around the lattice in direction mu is multiplied by bc[mu]: +1 periodic,
 * -1 antiperiodic, 0 open (the hop is dropped, so the lattice operator is
 * the Dirichlet operator of a block with these extents, paper Sec. 3).
 *
 * Memory: pointers named dev_* are device memory owned by the caller
 * (e.g. a torch tensor's data pointer); host_* are host memory.  Contexts
 * and gauge handles are owned by the library.  `stream` is a hipStream_t
 * (NULL = the default stream); every call is ordered on it.  Calls that
 * return host scalars (solve info, log ratios, samples to host) synchronise
 * the stream before returning.  A context (and its gauge handles) is used
 * by one host thread at a time: its workspace pool and solver read-back
 * buffers are not locked.
 *
 * Errors: no call throws.  Each returns a wdr_status; wdr_last_error()
 * gives a message for the calling thread.  A solver that reaches its
 * iteration limit returns WDR_ENOCONV with its outputs and info written.
 */
#ifndef WDR_H
#define WDR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WDR_OK = 0,
    WDR_EINVAL = -1,   /* invalid argument (geometry, kappa, pointer, size) */
    WDR_ENOMEM = -2,   /* device allocation failed */
    WDR_EDEVICE = -3,  /* a HIP call failed */
    WDR_ENOCONV = -4,  /* a solver stopped at max_iter above its tolerance */
    WDR_ESTATE = -5    /* handles that do not belong together */
} wdr_status;

typedef enum { WDR_F64 = 0, WDR_F32 = 1, WDR_F16 = 2 } wdr_prec;
typedef enum { WDR_NOISE_Z2 = 0, WDR_NOISE_GAUSS = 1 } wdr_noise_kind;

/* which determinant ratio is estimated (paper Sec. 3 eq. 4step, Sec. 4):
 * FULL   det(D'^+ D') / det(D^+ D)
 * SCHUR  det(Dhat'^+ Dhat') / det(Dhat^+ Dhat), Dhat = 1 - D_bb^-1 D_bw D_ww^-1 D_wb
 * BLOCKS det(D_b'^+ D_b') / det(D_b^+ D_b) for every block b separately
 * DD     the factorisation of eq. ddfactor: every BLOCKS ratio and the SCHUR
 *        ratio of one proposal in one call (one path; the two parts run
 *        concurrently); samples per (step, noise): nblocks block samples,
 *        then the Schur sample; the log ratio is their sum */
typedef enum { WDR_OP_FULL = 0, WDR_OP_SCHUR = 1, WDR_OP_BLOCKS = 2, WDR_OP_DD = 3 } wdr_op;

/* global solver: flexible GCR preconditioned by the Schwarz alternating
 * procedure, or CG on the normal equations D D^+ y = b, x = D^+ y */
typedef enum { WDR_SOLVER_FGCR_SAP = 0, WDR_SOLVER_CGNE = 1 } wdr_solver;

typedef struct {
    int32_t L[4];
    int32_t B[4];
    int32_t bc[4];
} wdr_geom;

typedef struct {
    wdr_solver solver;
    int32_t restart;     /* FGCR Krylov space before restart (16) */
    int32_t max_iter;    /* outer iterations (FGCR) or CG iterations */
    int32_t sap_cycles;  /* Schwarz cycles per preconditioner call (4) */
    int32_t mr_steps;    /* minimal-residual steps per block and cycle (5) */
    double tol;          /* ||b - D x|| / ||b|| of the global solves (1e-10) */
    double block_tol;    /* largest per-block relative residual of the
                            Dirichlet block solves (1e-13) */
    double adj_tol;      /* adjoint solves of the second-order sample (1e-7) */
    wdr_prec inner;      /* precision of the innermost level: the Schwarz
                            preconditioner (FGCR), the CG iterations (CGNE;
                            F16 = FP16 storage with per-block scales, the
                            FP16 stencil with its hops in packed FP16
                            arithmetic, FP32 updates) and the block MR */
    wdr_prec middle;     /* CGNE only: F64 = two levels (the CG iterations
                            in `inner` directly under the FP64 reliable
                            updates); F32 = three levels (inner = F16: FP16
                            iterations, FP32 reliable updates of the
                            iterated residual, FP64 reliable updates of the
                            solution with the true residual).  FGCR: F64 */
    int32_t block_mr_steps; /* MR steps per round of a defect-corrected block solve (16) */
    int32_t update_every;   /* CGNE steps between FP64 reliable-update / convergence points (4) */
    int32_t graph;          /* 1: CGNE replays each period of update_every steps as one HIP graph */
} wdr_solver_params;

typedef struct {
    int32_t iters;        /* outer iterations of the last solve */
    int32_t converged;    /* 1 if every solve met its tolerance */
    double true_rel_resid;/* FP64 ||b - D x|| / ||b|| of the last solve */
    double seconds;       /* wall time of the call */
    int64_t total_iters;  /* summed over all solves of the call */
} wdr_solve_info;

typedef struct {
    wdr_op op;
    int32_t n_steps;   /* N of eq. param: factors U_i -> U_{i+1}, i < N */
    int32_t n_noise;   /* independent noise vectors per factor */
    wdr_noise_kind noise;
    uint64_t seed;     /* Philox4x64-10 key (seed, 3) */
    wdr_solver_params sp;
    int32_t max_batch; /* most (proposal, step, noise) samples solved as the
                          systems of one batched pass; 0 = as many as fit */
} wdr_est_params;

/* One proposal U -> U' of wdr_logdet_ratio_batch. */
typedef struct {
    struct wdr_ctx *ctx;          /* context of the proposal's lattice */
    const struct wdr_gauge *U;    /* current links (a handle of ctx) */
    const struct wdr_gauge *Up;   /* proposed links (a handle of ctx) */
    double kappa;
    uint64_t seed;                /* noise key (seed, 3) of this proposal */
} wdr_proposal;

typedef struct wdr_ctx wdr_ctx;
typedef struct wdr_gauge wdr_gauge;

/* Message of the last error on the calling thread (never NULL). */
const char *wdr_last_error(void);
const char *wdr_status_str(wdr_status s);

/* Default solver parameters (FGCR(16)+SAP(4 cycles, 5 MR), tol 1e-10,
 * block_tol 1e-13, adj_tol 1e-7, FP32 inner, 16 MR steps per block-solve
 * round). */
void wdr_default_solver_params(wdr_solver_params *out);

/* Create a context for one lattice geometry on HIP device `device`.  Builds
 * the site ordering of Sec. 3 (black blocks first) and workspaces.
 * EINVAL for non-positive or non-dividing extents, odd B[mu], bc not in
 * {-1, 0, 1}. */
wdr_status wdr_ctx_create(const wdr_geom *geom, int device, wdr_ctx **out);
wdr_status wdr_ctx_destroy(wdr_ctx *ctx);

/* Number of sites V and block count of the context. */
int64_t wdr_ctx_volume(const wdr_ctx *ctx);
int32_t wdr_ctx_nblocks(const wdr_ctx *ctx);

/* Algorithmic device-memory traffic of the estimates of this process: the
 * compulsory bytes (every operand of a kernel read or written once; spinors
 * of the sites a kernel covers, each link and neighbour once) of the work
 * done by wdr_logdet_ratio / _batch and the solvers they call (CGNE and
 * the block solves, counted from their per-system iteration, update and
 * round counts; the FGCR / Schwarz solver is not counted), summed over all
 * contexts since the last reset.  reset = 1 returns the sum and clears it. */
int64_t wdr_traffic(int32_t reset);

/* Stencil kernel for the full operator D and the Dirichlet block operators
 * D_b (the hops of Sec. 3's blocks) on SU(3) fields with 4^4 blocks; the
 * result is the same operator either way, up to rounding order.
 * WDR_STENCIL_AUTO (the default): block-staged when a launch has at least
 * 2048 workgroups (blocks x systems), else direction-split.
 * WDR_STENCIL_DIR: direction-split (four workgroups per block, a wavefront
 * per direction).  WDR_STENCIL_BLK: block-staged (one workgroup per block,
 * the block's input read once into LDS).  Other operators (even-odd halves,
 * block-interaction hops) always use the direction-split kernel.  Applies to
 * later calls on ctx; EINVAL for another value. */
typedef enum { WDR_STENCIL_AUTO = 0, WDR_STENCIL_DIR = 1, WDR_STENCIL_BLK = 2 } wdr_stencil;
wdr_status wdr_ctx_set_stencil(wdr_ctx *ctx, int32_t choice);

/* Launch form of the FP32 and FP16 block MR of the Dirichlet block solves
 * (Sec. 3: the block operators D_b inverted inside the Schur complement of
 * eq. ddfactor) on 4^4 blocks; the arithmetic is the same either way.
 * WDR_MR_AUTO (the default): WDR_MR_TWO_PER_CU when a launch has at least
 * 2048 workgroups (blocks x systems), else WDR_MR_ONE_PER_CU.
 * WDR_MR_ONE_PER_CU: no register cap (one block per CU).
 * WDR_MR_TWO_PER_CU: compiled for four waves per SIMD (two blocks per CU,
 * some registers spilled).  Applies to later calls on ctx; EINVAL for
 * another value. */
typedef enum { WDR_MR_AUTO = 0, WDR_MR_ONE_PER_CU = 1, WDR_MR_TWO_PER_CU = 2 } wdr_mr_form;
wdr_status wdr_ctx_set_mr_form(wdr_ctx *ctx, int32_t choice);

/* Launch form of the CG steps of the even-odd CGNE with an F64 or F32 inner
 * level (the inversions of Sec. 4, "one inversion for each factor" of eq.
 * param); the arithmetic is the same either way, the inner products are
 * added in another order.  WDR_CG_LAUNCHES (the default): one kernel launch
 * per stencil half, reduction and update, about ten per step, captured as
 * HIP graphs with sp->graph.  WDR_CG_PERSISTENT: the sp->update_every steps
 * between two reliable updates run as one cooperative launch whose phases
 * are separated by grid-wide barriers (no graph capture); it applies to
 * 4^4 blocks with SU(3) links and no clover term, other solves keep the
 * launches.  The cooperative launch holds every resident workgroup slot of
 * the GPU it can use, so two of them must not run at once: the batched
 * estimate runs its contexts one after another when one of them has this
 * form, and the caller must not drive two such contexts of one GPU from two
 * threads.  EDEVICE from a solve whose cooperative launch the device
 * refuses.  Applies to later calls on ctx; EINVAL for another value. */
typedef enum { WDR_CG_LAUNCHES = 0, WDR_CG_PERSISTENT = 1 } wdr_cg_form;
wdr_status wdr_ctx_set_cg_form(wdr_ctx *ctx, int32_t choice);

/* Geometry maps (Sec. 3), written to caller device buffers of V int32:
 * block id (lexicographic block coordinates), block colour, site parity and
 * position of the site in the black-first block ordering. Any may be NULL. */
wdr_status wdr_site_maps(wdr_ctx *ctx, int32_t *dev_block_id, int32_t *dev_colour, int32_t *dev_parity,
                         int32_t *dev_position, void *stream);

/* Active-link mask (Sec. 3): for every block, the links with both ends in
 * the region of in-block coordinates [lo, hi]^4 and at most one end on the
 * boundary of that region (lo = 0, hi = B-1: whole blocks, Sec. 5; lo = 1,
 * hi = 6 in 8^4 blocks: the 6^4 core of Sec. 6).  dev_mask: V*4 uint8,
 * [site][mu] for the link x -> x+mu. */
wdr_status wdr_active_links(wdr_ctx *ctx, int32_t lo, int32_t hi, uint8_t *dev_mask, void *stream);

/* Upload a gauge field (canonical layout, dev_U device memory of V*4*9
 * complex).  The handle keeps FP64 and FP32 copies in the internal layout
 * with the boundary phases folded in. */
wdr_status wdr_gauge_create(wdr_ctx *ctx, const double *dev_U, wdr_gauge **out, void *stream);
wdr_status wdr_gauge_destroy(wdr_gauge *g);

/* 1 if every link of the uploaded field is SU(3) to 1e-10 (largest entry of
 * U U^+ - 1 and |det U - 1|), 0 otherwise or for a null handle.  SU(3)
 * fields let the stencil and the block solver read two rows per link and
 * rebuild the third (Sec. 5 uses SU(3) links throughout); other fields take
 * the paths that read all nine entries. */
int32_t wdr_gauge_is_su3(const wdr_gauge *g);

/* Attach the clover (Sheikholeslami-Wohlert) term to U: Sec. 3 defines the
 * active links for Wilson fermions with clover term and Sec. 7 names the
 * clover action.  The paper does not write the term out; it is the standard
 * one in the hopping normalisation of D = 1 - kappa H:
 *     D = A - kappa H,  A(x) = 1 + c_sw kappa (i/2) sum_{mu,nu} sigma_{mu nu} Fhat_{mu nu}(x),
 *     sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu],  Fhat_{mu nu} = (Q_{mu nu} - Q_{nu mu}) / 8,
 * Q_{mu nu}(x) the four plaquettes of the (mu, nu) plane at x (the clover
 * leaves).  The handle then keeps A and A^-1 (two hermitian 6 x 6 blocks per
 * site, FP64 and FP32: 1728 bytes per site) built for this csw and kappa, and
 * every call that takes U applies the clover operator: D, D_b and D_ee in F64
 * / F32 (wdr_apply_D, wdr_apply_D_internal, wdr_apply_D_noalloc,
 * wdr_apply_Dblock, wdr_apply_Dee; the hops of wdr_apply_Dhop have no
 * diagonal term), wdr_solve with CGNE or FGCR and wdr_sap (the Schwarz
 * blocks take the one-lane-per-site block MR; an F16 inner level sweeps in
 * F32 there, since the FP16 sweep keeps no blocks of A beside its fields),
 * wdr_block_solve and wdr_apply_schur (with an F64 / F32 inner level the
 * block solves then run as FP64 defect correction around an even-odd CGNE of
 * the block operator; with F16 the FP16 block MR keeps A_ee - 1 and A_oo^-1
 * of the block as FP16 in LDS), and FULL, BLOCKS, SCHUR and DD
 * estimates by such solves (wdr_logdet_ratio / _batch; both fields of a
 * ratio must carry the same csw), and the exact
 * block determinants (wdr_block_logdet / _ratio: det D_b = det A_oo det
 * Dhat_b with Dhat_b = A_ee - kappa^2 H_eo A_oo^-1 H_oe).  Those calls
 * must pass this kappa (EINVAL
 * otherwise); every other call taking U returns EINVAL.  csw = 0 removes the
 * term.  EINVAL also for a context with open boundaries (bc = 0) and when a
 * block of A is (nearly) singular (its LDL^H pivots are checked).  Waits for
 * the device: launches queued on U may still read the previous term. */
wdr_status wdr_gauge_set_clover(wdr_ctx *ctx, wdr_gauge *U, double csw, double kappa, void *stream);

/* A (inverse 0) or A^-1 (inverse 1) of U's clover term as canonical
 * [V][12][12] complex in device memory dev_out (row and column 3 * spin +
 * colour, chiral basis); EINVAL if U carries no clover term. */
wdr_status wdr_clover_field(wdr_ctx *ctx, const wdr_gauge *U, int32_t inverse, double *dev_out, void *stream);

/* Path of eq. param: out = U_i = exp((i/N) log(U' U^+)) U link by link
 * (geodesic with the traceless branch of the logarithm; U_0 = U and U_N = U'
 * exactly; links with U' == U copied). dev_out: canonical, V*4*9 complex. */
wdr_status wdr_interpolate(wdr_ctx *ctx, const double *dev_U, const double *dev_Up, int32_t i, int32_t N,
                           double *dev_out, void *stream);

/* Noise vector for path step `step`, sample k (paper Sec. 4: an independent
 * complex Gaussian noise vector for every factor of eq. param; black sites
 * only for the Schur complement, whose vectors live on the black blocks of
 * Sec. 3): for every site (all sites, or only black-block sites if
 * black_only), the words of
 * Philox4x64-10(counter = (site, step, k, j), key = (seed, 3)), j = 0..5,
 * give complex Gaussian components sqrt(-ln u) exp(2 pi i u') with
 * u = ((w >> 11) + 1/2) 2^-53 (E|eta|^2 = 1), or Z2 components
 * 1 - 2 * bit a of the first word. dev_out: canonical spinor. */
wdr_status wdr_noise(wdr_ctx *ctx, wdr_noise_kind kind, uint64_t seed, int32_t step, int32_t k, int32_t black_only,
                     double *dev_out, void *stream);

/* Internal layout (for callers that keep fields resident between calls):
 * one spinor field in precision prec (F64: complex double, F32: complex
 * float, F16: complex half) occupies wdr_field_bytes(ctx, prec) bytes of
 * device memory, ordered block by block (black blocks first, paper Sec. 3),
 * even sites before odd sites inside a block, component-major inside a
 * block.  An F16 field stores fp16(v / s_b) with one power-of-two scale s_b
 * >= max |component| per block (2^ceil(log2 max), 1 for a zero block); the
 * 12 V half-precision complex values are followed by the block scales (one
 * float per block, in block-slot order).  wdr_pack converts a canonical FP64
 * spinor to it (rounding to prec), wdr_unpack back. */
int64_t wdr_field_bytes(const wdr_ctx *ctx, wdr_prec prec);
wdr_status wdr_pack(wdr_ctx *ctx, wdr_prec prec, const double *dev_canon, void *dev_internal, void *stream);
wdr_status wdr_unpack(wdr_ctx *ctx, wdr_prec prec, const void *dev_internal, double *dev_canon, void *stream);

/* Halo of a lattice cut along t into slabs of whole blocks, one per GPU
 * (the sharding of a lattice too large for one GPU).  Sec. 3, eq. domdec:
 * D is its block-diagonal part plus the hops between blocks; the hops
 * between two slabs are block-interaction hops across the cut, and the rest
 * is the slab's own D with an open t boundary (wdr_apply_D_internal on a
 * context with bc[3] = 0; both calls below need such a context and EINVAL
 * otherwise).  Fields are internal-layout F64 or F32 fields of the slab (EINVAL
 * for F16); U is the slab's canonical FP64 links (the input of
 * wdr_gauge_create, device memory).  A face buffer holds one t slice's half
 * spinors, wdr_halo_bytes(ctx, prec) bytes: [6][F] complex of prec, F = L0
 * L1 L2 sites in the order x0 + L0 (x1 + L1 x2), components h0 then h1 of
 * the projected half spinor, colour fastest.
 *   wdr_halo_pack: send_lo = (1 - g_t) psi on the slice t = 0, for the slab
 *     below; send_hi = (1 + g_t) U_t^+ psi on the slice t = L3 - 1, for the
 *     slab above (the link lives on this slab).
 *   wdr_halo_unpack: out -= kappa [ sign_hi (1 - g_t) U_t(x) h on t = L3 - 1,
 *     h = recv_hi (the send_lo of the slab above); sign_lo (1 + g_t) c on
 *     t = 0, c = recv_lo (the send_hi of the slab below) ], the signs being
 *     the boundary condition of links that cross the lattice's time boundary
 *     (bc_t for the slabs at its two ends, else 1; 1 or -1, EINVAL otherwise).
 * The exchange itself (send_lo to the slab below, send_hi to the slab
 * above) is the caller's: one peer copy per face over xGMI.  Both calls
 * queue one kernel on `stream` and allocate nothing. */
int64_t wdr_halo_bytes(const wdr_ctx *ctx, wdr_prec prec);
wdr_status wdr_halo_pack(wdr_ctx *ctx, const double *dev_U, wdr_prec prec, const void *dev_in, void *dev_send_lo,
                         void *dev_send_hi, void *stream);
wdr_status wdr_halo_unpack(wdr_ctx *ctx, const double *dev_U, double kappa, wdr_prec prec, const void *dev_recv_lo,
                           const void *dev_recv_hi, int32_t sign_lo, int32_t sign_hi, void *dev_out, void *stream);

/* out = D in on internal-layout fields of precision prec: exactly one
 * stencil kernel launch on `stream`, no conversion.  F16 (arithmetic in
 * FP32, output rounded with its own block scales) needs 4^4 blocks and an
 * SU(3) gauge field (its links are the FP16 first two rows); otherwise
 * WDR_EINVAL. */
wdr_status wdr_apply_D_internal(wdr_ctx *ctx, const wdr_gauge *U, double kappa, wdr_prec prec,
                                const void *dev_in, void *dev_out, void *stream);

/* Even-odd halves on internal fields (the stencil of the even-odd CG of
 * wdr_solve; D = 1 - kappa H splits into the hops H_eo from odd to even
 * sites and H_oe from even to odd).  One call is exactly one kernel launch
 * on `stream`:
 *   out = diag - kappa H_{p, 1-p} in   on the sites of parity p = parity,
 * with gamma_5 H gamma_5 in place of H when dag = 1 (the half of D^+);
 * dev_diag may be NULL (no diagonal term); in, diag and out must not alias.
 * nsys systems share the gauge field U and sit back to back:
 *   F64 / F32: nsys fields of wdr_field_bytes(ctx, prec) bytes each; the
 *              sites of the other parity are read from in, written in
 *              out nowhere.
 *   F16:       the layout of the FP16 even-odd CG, which holds one parity
 *              of every block: nsys x wdr_eo16_field_bytes(ctx) bytes, all
 *              values first ([system][block slot][site of that parity in
 *              the in-block order][12] FP16 complex, 48 bytes per site),
 *              then one float power-of-two scale per (system, slot) >= the
 *              largest |component| of that block's half (stored value =
 *              value / scale); in holds parity 1 - p, diag and out parity p,
 *              and out receives fresh scales.  The hops are computed in
 *              packed FP16 on the stored values, each hop scaled and summed
 *              in FP32.  Needs 4^4 blocks in a 2-colourable checkerboard
 *              and an SU(3) field.
 * EINVAL otherwise. */
int64_t wdr_eo16_field_bytes(const wdr_ctx *ctx);
wdr_status wdr_apply_hop_eo_internal(wdr_ctx *ctx, const wdr_gauge *U, double kappa, wdr_prec prec, int32_t parity,
                                     int32_t dag, int32_t nsys, const void *dev_in, const void *dev_diag,
                                     void *dev_out, void *stream);
/* The sites of parity `parity` of a canonical spinor into one F16 half field
 * of that layout (scales from the block maxima), and back (the other
 * parity's sites of dev_canon set to zero). */
wdr_status wdr_pack_eo16(wdr_ctx *ctx, int32_t parity, const double *dev_canon, void *dev_eo16, void *stream);
wdr_status wdr_unpack_eo16(wdr_ctx *ctx, int32_t parity, const void *dev_eo16, double *dev_canon, void *stream);

/* out = D in (canonical spinors), computed in precision `prec` (F16 as for
 * wdr_apply_D_internal, input rounded by wdr_pack). */
wdr_status wdr_apply_D(wdr_ctx *ctx, const wdr_gauge *U, double kappa, wdr_prec prec, const double *dev_in,
                       double *dev_out, void *stream);

/* wdr_apply_D (F64 or F32) without any device allocation, for callers that
 * cannot allocate: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The two internal-layout staging fields
 * of a call live in a static device array of 64 MiB that each device the
 * library runs on holds until the process ends (its address is taken once
 * per device by wdr_ctx_create), so V x 12 complex of prec, twice, must fit:
 * at most 174762 sites in F64, 349525 in F32; EINVAL beyond.  Every call on
 * one device shares that array: calls that overlap on one GPU (on different
 * streams or host threads) race, and the caller must order them.  Results
 * equal wdr_apply_D's bit for bit. */
wdr_status wdr_apply_D_noalloc(wdr_ctx *ctx, const wdr_gauge *U, double kappa, wdr_prec prec, const double *dev_in,
                               double *dev_out, void *stream);

/* Dirichlet block operators (Sec. 3, eq. domdec): colour 0 gives D_bb,
 * 1 gives D_ww, 2 both; zero on sites outside the selected blocks. */
wdr_status wdr_apply_Dblock(wdr_ctx *ctx, const wdr_gauge *U, double kappa, wdr_prec prec, int32_t colour,
                            const double *dev_in, double *dev_out, void *stream);

/* Block-interaction hops (Sec. 3, eq. domdec: the off-diagonal blocks D_bw
 * and D_wb of D in the black/white block ordering, i.e. the hops that cross
 * a block face): from_colour 1 gives D_bw (white -> black sites), 0 gives
 * D_wb; zero on the sites of colour from_colour. */
wdr_status wdr_apply_Dhop(wdr_ctx *ctx, const wdr_gauge *U, double kappa, wdr_prec prec, int32_t from_colour,
                          const double *dev_in, double *dev_out, void *stream);

/* Even-odd reduced operator (1 - kappa^2 H_eo H_oe) on even sites, with all
 * hops (blocked = 0) or in-block hops only (blocked = 1); odd sites zero. */
wdr_status wdr_apply_Dee(wdr_ctx *ctx, const wdr_gauge *U, double kappa, wdr_prec prec, int32_t blocked,
                         const double *dev_in, double *dev_out, void *stream);

/* Schwarz alternating procedure: sp->sap_cycles cycles over black then white
 * blocks, each block updated by sp->mr_steps even-odd minimal-residual steps,
 * in precision sp->inner (F32 for F16 when U carries a clover term).  out
 * approximates D^-1 in. */
wdr_status wdr_sap(wdr_ctx *ctx, const wdr_gauge *U, double kappa, const wdr_solver_params *sp,
                   const double *dev_in, double *dev_out, void *stream);

/* Solve D x = b to sp->tol (true FP64 residual): the inversion that Sec. 4
 * needs once for each factor of eq. param (D of the proposed field U_{i+1}).
 * Either solver of sp->solver, at the precisions of sp->inner / sp->middle;
 * info (host, may be NULL): iterations and the true residual.  ENOCONV at
 * sp->max_iter with x and info written. */
wdr_status wdr_solve(wdr_ctx *ctx, const wdr_gauge *U, double kappa, const wdr_solver_params *sp,
                     const double *dev_b, double *dev_x, wdr_solve_info *host_info, void *stream);

/* Solve the Dirichlet block systems of one colour (2: all blocks) to
 * sp->block_tol (Sec. 3, eq. domdec: D_bb and D_ww are block diagonal with
 * the Dirichlet block operators D_b on the diagonal, so their inverses in
 * eq. ddfactor are independent block solves): x = D_cc^-1 b on those blocks,
 * zero elsewhere; per-block relative residual <= block_tol.  Even-odd MR
 * rounds in sp->inner with FP64 defect correction (with a clover term and
 * sp->inner F64 or F32: rounds of even-odd CGNE on the blocks of the
 * colour).  ENOCONV if a block stops above block_tol. */
wdr_status wdr_block_solve(wdr_ctx *ctx, const wdr_gauge *U, double kappa, int32_t colour,
                           const wdr_solver_params *sp, const double *dev_b, double *dev_x,
                           wdr_solve_info *host_info, void *stream);

/* Schur complement (Sec. 3, eq. ddfactor): out = Dhat in
 * = in - D_bb^-1 D_bw D_ww^-1 D_wb in on black sites (white sites of in
 * ignored, of out zero); block solves to sp->block_tol. */
wdr_status wdr_apply_schur(wdr_ctx *ctx, const wdr_gauge *U, double kappa, const wdr_solver_params *sp,
                           const double *dev_in, double *dev_out, void *stream);

/* Stochastic estimate of the log determinant ratio for U -> U' (Sec. 4):
 * for i < n_steps and k < n_noise, with U_i from the path of eq. param and
 * eta_{i,k} from wdr_noise (black sites for SCHUR), the sample
 *   s_{i,k} = -eta^+ (M_i^+ M_i - 1) eta,  M_i = X(U_{i+1})^-1 X(U_i),
 * evaluated to second order in the solver residual.  host_samples receives
 * n_steps*n_noise values ([i][k]), times nblocks for BLOCKS ([i][k][block])
 * and nblocks + 1 for DD ([i][k][block], then the Schur sample);
 * *host_log_ratio = sum_i log((1/n_noise) sum_k exp(s_{i,k})) (for BLOCKS
 * the sum over blocks).  Either output pointer may be NULL. */
wdr_status wdr_logdet_ratio(wdr_ctx *ctx, const wdr_gauge *U, const wdr_gauge *Up, double kappa,
                            const wdr_est_params *p, double *host_samples, double *host_log_ratio,
                            wdr_solve_info *host_info, void *stream);

/* The estimate of wdr_logdet_ratio for n independent proposals (possibly on
 * lattices of different sizes) in one batched pass (Sec. 4, eq. param: the
 * factors of one proposal, and separate proposals, are independent given
 * their paths and noise keys, so every factor is an independent system).  Proposals that share a
 * context are solved together: every (proposal, step, noise) sample is one
 * system of the same launches, with its own links, kappa and noise key
 * (props[j].seed; p->seed is not used).  Groups on different contexts run
 * concurrently, each on a stream of its context ordered after `stream`;
 * the call returns when all are done.  host_samples: the proposals in order,
 * each n_steps*n_noise values (times the nblocks of its context for BLOCKS);
 * host_log_ratios: n values; host_info: summed iterations, the worst
 * residual over all solves.  Proposals of one context must all use SU(3)
 * links or none do (mixing only costs speed).  A context may appear in one
 * call at a time and no other call may use it meanwhile. */
wdr_status wdr_logdet_ratio_batch(int32_t n, const wdr_proposal *props, const wdr_est_params *p,
                                  double *host_samples, double *host_log_ratios, wdr_solve_info *host_info,
                                  void *stream);

/* Schedule autotuner for wdr_logdet_ratio on this context: times a short
 * estimate (at most eight path factors, the noise key of *p plus one; the
 * faster of two runs after a warm-up run) for a set of Schwarz depths
 * (cycles x MR steps, FGCR only), then of block-solve MR depths (ratios with
 * block solves), then of launch forms (the block-MR form of
 * wdr_ctx_set_mr_form, then the stencil kernel of wdr_ctx_set_stencil), and
 * writes the fastest depths into p->sp and the fastest forms into the
 * context (as the two setters would).  Every candidate solves to the
 * tolerances of p->sp, so the choice changes time only.  The result is
 * cached in the context per (ratio, solver, inner and middle precision,
 * kappa); a cached result restores its forms.  host_seconds (may be NULL)
 * receives the time of the chosen candidate. */
wdr_status wdr_autotune(wdr_ctx *ctx, const wdr_gauge *U, const wdr_gauge *Up, double kappa, wdr_est_params *p,
                        double *host_seconds, void *stream);

/* Exact block factors of eq. ddfactor (paper Sec. 3): host_out[b] =
 * log det(D_b^+ D_b) of the Dirichlet block operator D_b (in-block hops
 * only) of every block b, indexed by lexicographic block id (nblocks
 * doubles).  Their differences between U' and U are the exact block ratios
 * of the first acceptance step of eq. 4step.  Computed in FP64 on the
 * device: the even-odd reduced normal matrix Dhat_b^+ Dhat_b (6 Vb rows,
 * det D_b = det Dhat_b) of each block is formed and Cholesky-factorised;
 * the result is 2 sum log L_ii.  Workspace: 16 (6 Vb rounded up to a
 * multiple of 64)^2 bytes per block matrix (with a clover term on U, see
 * wdr_gauge_set_clover, the term enters Dhat_b and log det A_oo of the odd
 * sites is added); the matrices are factorised in
 * passes of max_blocks (0: as many as fit in 8 GiB).  Returns after the
 * stream has finished.  EINVAL for blocks of more than 256 sites
 * or L/B odd in some direction; ENOCONV if a factorisation met a
 * non-positive pivot (D_b singular to FP64 precision): those entries are
 * NaN, the others valid. */
wdr_status wdr_block_logdet(wdr_ctx *ctx, const wdr_gauge *U, double kappa, int32_t max_blocks, double *host_out,
                            void *stream);

/* host_out[b] = log det(D_b'^+ D_b') - log det(D_b^+ D_b): the exact block
 * ratios between U' and U (eq. 4step, first step), the matrices of both
 * fields in one batch.  Errors as wdr_block_logdet. */
wdr_status wdr_block_logdet_ratio(wdr_ctx *ctx, const wdr_gauge *U, const wdr_gauge *Up, double kappa,
                                  int32_t max_blocks, double *host_out, void *stream);

/* Links of every block of ctx as a lattice of its own: dev_out[b] (b by
 * lexicographic block id) is a canonical gauge field of extents B (the
 * block's sites in lexicographic order, all four links of each site, the
 * links leaving the block included), nblocks x V_b x 36 complex.  The
 * boundary phases of ctx are not applied.  For a context with extents B and
 * open boundaries these are the fields whose lattice operator is each
 * block's Dirichlet operator D_b (Sec. 3). */
wdr_status wdr_block_fields(wdr_ctx *ctx, const wdr_gauge *U, double *dev_out, void *stream);

/* Recursive domain decomposition (Sec. 3, eq. ddrec; the block step 2 of
 * eq. 4step): for every block b of ctx, the stochastic estimate of
 *     log det(Dhat_b'^+ Dhat_b') / det(Dhat_b^+ Dhat_b),
 * Dhat_b the Schur complement of the Dirichlet block operator D_b over
 * sub-blocks.  `sub` describes one block: L = the blocks' extents of ctx,
 * bc = 0 in every direction, B = the sub-block extents.  All blocks are
 * estimated in one batched call on `sub` (wdr_logdet_ratio_batch with
 * op WDR_OP_SCHUR, which p->op must be); block b uses the noise key
 * p->seed + b.  host_samples: nblocks x n_steps x n_noise; host_log_ratios:
 * nblocks; host_info: summed iterations, worst residual.  Needs SU(3) links
 * or none in both fields; EINVAL for a mismatched `sub`, and for fields that
 * carry a clover term (the clover leaves at a block's faces reach links
 * outside the block, which `sub` does not hold). */
wdr_status wdr_block_schur_ratio(wdr_ctx *ctx, const wdr_gauge *U, const wdr_gauge *Up, double kappa, wdr_ctx *sub,
                                 const wdr_est_params *p, double *host_samples, double *host_log_ratios,
                                 wdr_solve_info *host_info, void *stream);

/* Heat-bath sweep of the links marked in dev_mask (V x 4 bytes, entry
 * 4 site + mu, canonical site order) of the canonical field dev_U, in place,
 * for the Wilson plaquette action beta sum_P (1 - Re tr U_P / 3) (paper
 * Sec. 5; the gauge update of step 0 of eq. 4step).  Directions mu = 0..3,
 * within each the sites of even then odd parity; each link takes the
 * Cabibbo-Marinari steps over the SU(2) subgroups (0,1), (0,2), (1,2) with
 * Kennedy-Pendleton sampling.  Random numbers: Philox4x64-10, key (seed, 5),
 * counter (site, sweep 2^32 + mu 2^8 + subgroup, trial, j), uniforms
 * ((w >> 11) + 1/2) 2^-53; j = 0 holds the four uniforms of a trial, j = 1
 * the direction of the accepted one; a subgroup that rejects 64 trials
 * stays unchanged.  Plaquettes are periodic whatever bc. */
wdr_status wdr_heatbath(wdr_ctx *ctx, double beta, const uint8_t *dev_mask, uint64_t seed, int32_t sweep,
                        double *dev_U, void *stream);

/* Over-relaxation sweep of the masked links (the alternative that Sec. 5
 * names beside the heat-bath), in the order of wdr_heatbath: per SU(2)
 * subgroup, with the subgroup part of W = U A equal to k v (v in SU(2)),
 * U <- (v^+)^2 U, which keeps the Wilson action.  No random numbers. */
wdr_status wdr_overrelax(wdr_ctx *ctx, const uint8_t *dev_mask, double *dev_U, void *stream);

/* Relative gauge fixing of the canonical field dev_Up to dev_U, in place
 * (paper Sec. 4: it narrows the spectrum of M^+ M, M = X'^-1 X): `sweeps`
 * sweeps of local maximisation of F = sum_{x,mu} Re tr(U'_mu(x) U_mu(x)^+)
 * over gauge transformations of U', even then odd sites.  At site x the
 * transformation h is built from the identity by one pass over the SU(2)
 * subgroups (0,1), (0,2), (1,2) maximising Re tr(h K),
 * K = sum_mu [U'_mu(x) U_mu(x)^+ + U'_mu(x-mu)^+ U_mu(x-mu)].  Every
 * determinant of the operators here is gauge invariant; the path U -> U'
 * and so the estimator's variance change.  Periodic in every direction
 * (a gauge transformation ignores bc).  host_F (may be NULL): F / 3 after
 * the sweeps. */
wdr_status wdr_relative_gauge(wdr_ctx *ctx, const double *dev_U, double *dev_Up, int32_t sweeps, double *host_F,
                              void *stream);

typedef struct wdr_filter_info {
    int32_t block_accepts; /* accepted blocks, summed over the block steps */
    int32_t block_trials;  /* n_block_steps x nblocks */
    int32_t accepted;      /* the global step accepted the result */
    int32_t pad;
    double log_ratio;      /* the global estimate log Rhat */
} wdr_filter_info;

/* One step of the hierarchical filter, eq. 4step with one level (the
 * three-step algorithm of paper Sec. 5), on the canonical field dev_U in
 * place.  n_block_steps times: a heat-bath sweep of the masked links (sweep
 * index = step), then each block accepted with probability
 * min(1, exp(r_b)), r_b = log det(D_b'^+ D_b') - log det(D_b^+ D_b) from the
 * exact block determinants (uniform from Philox key (seed, 6), counter
 * (block, step, 0, 0)); rejected blocks keep their links.  Then the result
 * is accepted with probability min(1, exp(log Rhat)), log Rhat the estimate
 * of *p (op WDR_OP_SCHUR) from the field before the step to the result
 * (uniform from counter (0, 0, 1, 0)); a rejected step restores dev_U.
 * p = NULL runs the block steps only and keeps their result (the proposal
 * the global step would decide on).  host_accepts (NULL allowed):
 * n_block_steps x nblocks block decisions.
 * EINVAL if the mask holds a link that leaves its block. */
wdr_status wdr_filter_step(wdr_ctx *ctx, double beta, double kappa, const uint8_t *dev_mask, int32_t n_block_steps,
                           const wdr_est_params *p, uint64_t seed, double *dev_U, uint8_t *host_accepts,
                           wdr_filter_info *host_info, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* WDR_H */
