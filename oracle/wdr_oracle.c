/*
 * wdr_oracle.c -- plain, slow, FP64 CPU oracle for the Wilson-Dirac
 * determinant-ratio path of Leder, Finkenrath and Knechtli, "Fermions as
 * global correction in lattice QCD" (Lattice 2011).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or constant with the HIP library.
 *
 * Everything works on the canonical layout:
 *   site  = x0 + L0*(x1 + L1*(x2 + L2*x3))
 *   psi   [site][spin 4][colour 3]        (double complex)
 *   U     [site][mu 4][row 3][col 3]      (double complex), U_mu(x) is the
 *         link from x to x+mu.
 *
 * Operator (the "plain Wilson-Dirac operator" with hopping parameter kappa,
 * paper Sec. 5; sign and basis conventions are this project's reading):
 *   (D psi)(x) = psi(x) - kappa * sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
 *                                        + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu) ]
 * with the spin matrices applied as full 4x4 matrices (no projection trick).
 * A hop that wraps around the lattice in direction mu is multiplied by bc[mu].
 *
 * With the clover term (Sheikholeslami-Wohlert; Sec. 3 names Wilson fermions
 * with clover term, Sec. 7 the clover action) the diagonal 1 becomes 1 + T(x),
 * T(x) a 12 x 12 matrix per site built in core.py from its definition and
 * passed in as clov[site][12][12] (row 3*spin + colour); NULL means no term.
 *
 * Domain decomposition (paper Sec. 3, eq. domdec): non-overlapping blocks of
 * extent B[mu]; the block colour is (sum_mu floor(x_mu/B_mu)) mod 2, black =
 * 0.  D_b keeps only hops whose both ends lie in block b (Dirichlet
 * boundaries); the interaction terms D_bw, D_wb keep only the hops that cross
 * a block boundary.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* small lattices run serially: waking threads costs more than the work */
#define OMP_MIN_SITES 8192

/* ------------------------------------------------------------------ */
/* Dirac matrices: chiral basis, lattice mu = 0,1,2 -> gamma_1,2,3 and
 * mu = 3 -> gamma_4.  gamma_k = [[0, -i s_k], [i s_k, 0]],
 * gamma_4 = [[0, 1], [1, 0]], so gamma_5 = g1 g2 g3 g4 = diag(1,1,-1,-1). */
static const cplx GAMMA[4][4][4] = {
    /* gamma_1 */
    {{0, 0, 0, -I}, {0, 0, -I, 0}, {0, I, 0, 0}, {I, 0, 0, 0}},
    /* gamma_2 */
    {{0, 0, 0, -1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {-1, 0, 0, 0}},
    /* gamma_3 */
    {{0, 0, -I, 0}, {0, 0, 0, I}, {I, 0, 0, 0}, {0, -I, 0, 0}},
    /* gamma_4 */
    {{0, 0, 1, 0}, {0, 0, 0, 1}, {1, 0, 0, 0}, {0, 1, 0, 0}},
};

void oracle_gamma(int mu, double *out /* 4x4 complex, row-major */)
{
    for (int s = 0; s < 4; ++s)
        for (int t = 0; t < 4; ++t) {
            out[2 * (4 * s + t)] = creal(GAMMA[mu][s][t]);
            out[2 * (4 * s + t) + 1] = cimag(GAMMA[mu][s][t]);
        }
}

/* ------------------------------------------------------------------ */
/* Geometry */

typedef struct {
    int L[4];
    int B[4];
    int bc[4];
    long V;
} geom_t;

static geom_t make_geom(const int *L, const int *B, const int *bc)
{
    geom_t g;
    g.V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        g.L[mu] = L[mu];
        g.B[mu] = B ? B[mu] : L[mu];
        g.bc[mu] = bc ? bc[mu] : 1;
        g.V *= L[mu];
    }
    return g;
}

static void coords(const geom_t *g, long s, int x[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        x[mu] = (int)(s % g->L[mu]);
        s /= g->L[mu];
    }
}

static long index_of(const geom_t *g, const int x[4])
{
    return x[0] + (long)g->L[0] * (x[1] + (long)g->L[1] * (x[2] + (long)g->L[2] * x[3]));
}

static int colour_of(const geom_t *g, const int x[4])
{
    int c = 0;
    for (int mu = 0; mu < 4; ++mu) c += x[mu] / g->B[mu];
    return c & 1;
}

static int parity_of(const int x[4]) { return (x[0] + x[1] + x[2] + x[3]) & 1; }

static int same_block(const geom_t *g, const int x[4], const int y[4])
{
    for (int mu = 0; mu < 4; ++mu)
        if (x[mu] / g->B[mu] != y[mu] / g->B[mu]) return 0;
    return 1;
}

static long block_lex(const geom_t *g, const int x[4])
{
    long b = 0;
    for (int mu = 3; mu >= 0; --mu) b = b * (g->L[mu] / g->B[mu]) + x[mu] / g->B[mu];
    return b;
}

/* neighbour of x in direction mu, forward (dir=+1) or backward (dir=-1);
 * returns the boundary phase (bc[mu] if the hop wraps, else 1). */
static int neighbour(const geom_t *g, const int x[4], int mu, int dir, int y[4])
{
    int phase = 1;
    for (int nu = 0; nu < 4; ++nu) y[nu] = x[nu];
    y[mu] += dir;
    if (y[mu] == g->L[mu]) { y[mu] = 0; phase = g->bc[mu]; }
    if (y[mu] < 0) { y[mu] = g->L[mu] - 1; phase = g->bc[mu]; }
    return phase;
}

/* block id, colour, parity for every canonical site */
void oracle_site_maps(const int *L, const int *B, int32_t *block_id, int32_t *colour, int32_t *parity)
{
    geom_t g = make_geom(L, B, NULL);
    for (long s = 0; s < g.V; ++s) {
        int x[4];
        coords(&g, s, x);
        block_id[s] = (int32_t)block_lex(&g, x);
        colour[s] = colour_of(&g, x);
        parity[s] = parity_of(x);
    }
}

/* ------------------------------------------------------------------ */
/* Generic hopping operator.
 *
 *   out(x) = diag * (1 + T(x)) in(x) - kappa * sum over selected hops (x <- y)
 *
 * with T = 0 when clov is NULL.
 * selection:
 *   hops      0 = every hop, 1 = only hops inside a block, 2 = only hops
 *             that cross a block boundary
 *   out_col   output only on sites of this block colour (-1: all); other
 *             sites get zero
 *   in_col    take the input only from sites of this colour (-1: all)
 *   out_par   output only on sites of this parity (-1: all)
 *   in_par    take the input only from sites of this parity (-1: all)
 */
enum { HOPS_ALL = 0, HOPS_IN_BLOCK = 1, HOPS_CROSS = 2 };

static void wilson_generic(const geom_t *g, double kappa, const cplx *U, const cplx *clov, const cplx *in,
                           cplx *out, int diag, int hops, int out_col, int in_col, int out_par, int in_par)
{
#pragma omp parallel for schedule(static) if (g->V >= OMP_MIN_SITES)
    for (long s = 0; s < g->V; ++s) {
        int x[4];
        coords(g, s, x);
        cplx acc[4][3];
        if ((out_col >= 0 && colour_of(g, x) != out_col) || (out_par >= 0 && parity_of(x) != out_par)) {
            for (int a = 0; a < 12; ++a) out[12 * s + a] = 0;
            continue;
        }
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) acc[sp][a] = diag ? in[12 * s + 3 * sp + a] : 0;
        if (diag && clov) {
            const cplx *Tx = clov + 144 * s;
            for (int i = 0; i < 12; ++i)
                for (int j = 0; j < 12; ++j) acc[i / 3][i % 3] += Tx[12 * i + j] * in[12 * s + j];
        }

        for (int mu = 0; mu < 4; ++mu) {
            for (int dir = +1; dir >= -1; dir -= 2) {
                int y[4];
                int phase = neighbour(g, x, mu, dir, y);
                int inside = same_block(g, x, y);
                if (hops == HOPS_IN_BLOCK && !inside) continue;
                if (hops == HOPS_CROSS && inside) continue;
                if (in_col >= 0 && colour_of(g, y) != in_col) continue;
                if (in_par >= 0 && parity_of(y) != in_par) continue;
                long t = index_of(g, y);
                const cplx *psi = in + 12 * t;
                /* colour multiply: chi_{sp,a} = sum_b W_ab psi_{sp,b},
                 * W = U_mu(x) forward, W = U_mu(x-mu)^+ backward */
                cplx chi[4][3];
                for (int sp = 0; sp < 4; ++sp)
                    for (int a = 0; a < 3; ++a) {
                        cplx v = 0;
                        for (int b = 0; b < 3; ++b) {
                            cplx w;
                            if (dir > 0) w = U[(36 * s) + 9 * mu + 3 * a + b];
                            else w = conj(U[(36 * t) + 9 * mu + 3 * b + a]);
                            v += w * psi[3 * sp + b];
                        }
                        chi[sp][a] = v;
                    }
                /* spin matrix (1 - dir * gamma_mu) */
                for (int sp = 0; sp < 4; ++sp)
                    for (int a = 0; a < 3; ++a) {
                        cplx v = 0;
                        for (int tp = 0; tp < 4; ++tp) {
                            cplx m = (sp == tp ? 1.0 : 0.0) - dir * GAMMA[mu][sp][tp];
                            v += m * chi[tp][a];
                        }
                        acc[sp][a] -= kappa * phase * v;
                    }
            }
        }
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) out[12 * s + 3 * sp + a] = acc[sp][a];
    }
}

/* full D (clov: clover term or NULL) */
void oracle_apply_D(const int *L, const int *bc, double kappa, const double *U, const double *clov, const double *in,
                    double *out)
{
    geom_t g = make_geom(L, NULL, bc);
    wilson_generic(&g, kappa, (const cplx *)U, (const cplx *)clov, (const cplx *)in, (cplx *)out, 1, HOPS_ALL, -1,
                   -1, -1, -1);
}

/* block-diagonal Dirichlet operator on the blocks of one colour (0 black,
 * 1 white, 2 both); zero on the sites of the other colour. */
void oracle_apply_Dblock(const int *L, const int *B, const int *bc, double kappa, const double *U,
                         const double *clov, int colour, const double *in, double *out)
{
    geom_t g = make_geom(L, B, bc);
    wilson_generic(&g, kappa, (const cplx *)U, (const cplx *)clov, (const cplx *)in, (cplx *)out, 1, HOPS_IN_BLOCK,
                   colour == 2 ? -1 : colour, -1, -1, -1);
}

/* block-interaction hops from the sites of one colour to the other:
 * from_colour = 1 gives D_bw (white -> black), 0 gives D_wb. */
void oracle_apply_Dhop(const int *L, const int *B, const int *bc, double kappa, const double *U, int from_colour,
                       const double *in, double *out)
{
    geom_t g = make_geom(L, B, bc);
    wilson_generic(&g, kappa, (const cplx *)U, NULL, (const cplx *)in, (cplx *)out, 0, HOPS_CROSS, 1 - from_colour,
                   from_colour, -1, -1);
}

/* even-odd reduced operator (1 - kappa^2 H_eo H_oe) psi_e, on the whole
 * lattice (blocked = 0) or with in-block hops only (blocked = 1).
 * Odd sites of the output are zero. */
void oracle_apply_Dee(const int *L, const int *B, const int *bc, double kappa, const double *U, int blocked,
                      const double *in, double *out)
{
    geom_t g = make_geom(L, B, bc);
    long n = 12 * g.V;
    cplx *t = calloc(n, sizeof(cplx));
    cplx *u = calloc(n, sizeof(cplx));
    int hops = blocked ? HOPS_IN_BLOCK : HOPS_ALL;
    /* t = -kappa H_oe psi_e ; u = -kappa H_eo t = kappa^2 H_eo H_oe psi_e */
    wilson_generic(&g, kappa, (const cplx *)U, NULL, (const cplx *)in, t, 0, hops, -1, -1, 1, 0);
    wilson_generic(&g, kappa, (const cplx *)U, NULL, t, u, 0, hops, -1, -1, 0, 1);
    const cplx *psi = (const cplx *)in;
    cplx *o = (cplx *)out;
    for (long s = 0; s < g.V; ++s) {
        int x[4];
        coords(&g, s, x);
        for (int a = 0; a < 12; ++a) o[12 * s + a] = parity_of(x) == 0 ? psi[12 * s + a] - u[12 * s + a] : 0;
    }
    free(t);
    free(u);
}

/* gamma_5 = diag(1,1,-1,-1) in spin */
static void mul_g5(long V, const cplx *in, cplx *out)
{
    for (long s = 0; s < V; ++s)
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) out[12 * s + 3 * sp + a] = (sp < 2 ? 1.0 : -1.0) * in[12 * s + 3 * sp + a];
}

void oracle_mul_g5(long V, const double *in, double *out) { mul_g5(V, (const cplx *)in, (cplx *)out); }

/* ------------------------------------------------------------------ */
/* Linear algebra helpers */

static cplx dot(long n, const cplx *a, const cplx *b) /* a^+ b */
{
    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) if (n >= 12 * OMP_MIN_SITES)
    for (long i = 0; i < n; ++i) {
        cplx v = conj(a[i]) * b[i];
        re += creal(v);
        im += cimag(v);
    }
    return re + I * im;
}

static double norm2(long n, const cplx *a) { return creal(dot(n, a, a)); }

/* operator selector for the solver: op 0 = full D, op 1 = Dirichlet blocks
 * of colour `colour` (0, 1 or 2 = both) */
typedef struct {
    const geom_t *g;
    double kappa;
    const cplx *U, *clov;
    int op, colour;
} opdesc_t;

static void op_apply(const opdesc_t *o, const cplx *in, cplx *out)
{
    if (o->op == 0)
        wilson_generic(o->g, o->kappa, o->U, o->clov, in, out, 1, HOPS_ALL, -1, -1, -1, -1);
    else
        wilson_generic(o->g, o->kappa, o->U, o->clov, in, out, 1, HOPS_IN_BLOCK, o->colour == 2 ? -1 : o->colour,
                       -1, -1, -1);
}

/* A^+ = g5 A g5 (gamma_5-hermiticity of the Wilson operator and of its
 * Dirichlet block restriction; the clover term is hermitian and commutes
 * with gamma_5, so it keeps the property) */
static void op_apply_dag(const opdesc_t *o, const cplx *in, cplx *out, cplx *tmp)
{
    mul_g5(o->g->V, in, tmp);
    op_apply(o, tmp, out);
    mul_g5(o->g->V, out, out);
}

/*
 * Solve A x = b by the conjugate-gradient method on the normal equations
 * A A^+ y = b, x = A^+ y.  Stops when the true residual ||b - A x|| / ||b||
 * is at most tol (the recursive residual is replaced by the true one at
 * every apparent convergence).  Returns the iteration count, or -1 if
 * maxit was reached.  On return y holds the normal-equation solution, x =
 * A^+ y and *rel_resid the true relative residual.
 */
int oracle_cgne(const int *L, const int *B, const int *bc, double kappa, const double *Ud, const double *clov, int op,
                int colour, const double *bd, double *xd, double *yd, double tol, int maxit, double *rel_resid)
{
    geom_t g = make_geom(L, B, bc);
    opdesc_t o = {&g, kappa, (const cplx *)Ud, (const cplx *)clov, op, colour};
    long n = 12 * g.V;
    const cplx *b = (const cplx *)bd;
    cplx *x = (cplx *)xd, *y = (cplx *)yd;
    cplx *r = malloc(n * sizeof(cplx)), *p = malloc(n * sizeof(cplx));
    cplx *q = malloc(n * sizeof(cplx)), *w = malloc(n * sizeof(cplx)), *tmp = malloc(n * sizeof(cplx));
    double bb = norm2(n, b);
    int it = 0, converged = 0;
    for (long i = 0; i < n; ++i) y[i] = 0, r[i] = b[i], p[i] = b[i];
    double rr = bb;
    if (bb == 0) {
        for (long i = 0; i < n; ++i) x[i] = 0;
        *rel_resid = 0;
        goto done_ok;
    }
    while (it < maxit) {
        /* q = A A^+ p */
        op_apply_dag(&o, p, w, tmp);
        op_apply(&o, w, q);
        double pq = creal(dot(n, p, q));
        double alpha = rr / pq;
        for (long i = 0; i < n; ++i) y[i] += alpha * p[i], r[i] -= alpha * q[i];
        double rr_new = norm2(n, r);
        ++it;
        if (rr_new <= tol * tol * bb * 0.25) {
            /* true residual of A x = b with x = A^+ y */
            op_apply_dag(&o, y, x, tmp);
            op_apply(&o, x, w);
            for (long i = 0; i < n; ++i) r[i] = b[i] - w[i];
            rr_new = norm2(n, r);
            if (rr_new <= tol * tol * bb) {
                converged = 1;
                rr = rr_new;
                break;
            }
            /* restart the direction from the true residual */
            for (long i = 0; i < n; ++i) p[i] = r[i];
            rr = rr_new;
            continue;
        }
        double beta = rr_new / rr;
        for (long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rr = rr_new;
    }
    op_apply_dag(&o, y, x, tmp);
    op_apply(&o, x, w);
    for (long i = 0; i < n; ++i) r[i] = b[i] - w[i];
    *rel_resid = sqrt(norm2(n, r) / bb);
    if (!converged && *rel_resid > tol) it = -1;
done_ok:
    free(r);
    free(p);
    free(q);
    free(w);
    free(tmp);
    return it;
}

/* ------------------------------------------------------------------ */
/* Schwarz alternating procedure (domain-decomposition preconditioner of
 * Luscher, hep-lat/0310048, cited by the paper in Secs. 1 and 3).
 *
 *   x = 0
 *   repeat ncy times, for colour c = black, white:
 *       r = eta - D x               on the blocks of colour c
 *       on every block b of colour c: delta_b = nmr minimal-residual steps
 *           for D_b delta_b = r_b, on the even-odd reduced block system
 *       x += delta
 *
 * Minimal residual on the reduced block system (D_b = A - kappa H_b, A = 1
 * without a clover term, A = 1 + T with one):
 *   rhs_e = r_e + kappa H_eo A_oo^-1 r_o
 *   d_e = 0, rho = rhs_e; nmr times: p = (A_ee - kappa^2 H_eo A_oo^-1 H_oe) rho,
 *       alpha_b = <p, rho>_b / <p, p>_b, d_e += alpha_b rho, rho -= alpha_b p
 *   d_o = A_oo^-1 (r_o + kappa H_oe d_e)
 * where H are the in-block (Dirichlet) hops and <.,.>_b sums over block b.
 */

/* (1 + T(x))^-1 of every site (144 complex each), by Gauss-Jordan
 * elimination with partial pivoting on [A | 1] */
static cplx *clover_inverse(const geom_t *g, const cplx *clov)
{
    cplx *inv = malloc(144 * g->V * sizeof(cplx));
    for (long s = 0; s < g->V; ++s) {
        cplx a[12][24];
        for (int i = 0; i < 12; ++i)
            for (int j = 0; j < 24; ++j)
                a[i][j] = j < 12 ? clov[144 * s + 12 * i + j] + (i == j ? 1.0 : 0.0) : (j - 12 == i ? 1.0 : 0.0);
        for (int k = 0; k < 12; ++k) {
            int piv = k;
            for (int i = k + 1; i < 12; ++i)
                if (cabs(a[i][k]) > cabs(a[piv][k])) piv = i;
            for (int j = 0; j < 24; ++j) {
                cplx tmp = a[k][j];
                a[k][j] = a[piv][j];
                a[piv][j] = tmp;
            }
            cplx f = 1.0 / a[k][k];
            for (int j = 0; j < 24; ++j) a[k][j] *= f;
            for (int i = 0; i < 12; ++i) {
                if (i == k) continue;
                cplx m = a[i][k];
                for (int j = 0; j < 24; ++j) a[i][j] -= m * a[k][j];
            }
        }
        for (int i = 0; i < 12; ++i)
            for (int j = 0; j < 12; ++j) inv[144 * s + 12 * i + j] = a[i][12 + j];
    }
    return inv;
}

/* v <- M(x) v on the sites of this colour and parity, M per site (144 complex) */
static void site_mul(const geom_t *g, const cplx *M, cplx *v, int colour, int par)
{
    for (long s = 0; s < g->V; ++s) {
        int x[4];
        coords(g, s, x);
        if (colour_of(g, x) != colour || parity_of(x) != par) continue;
        cplx w[12];
        for (int i = 0; i < 12; ++i) {
            w[i] = 0;
            for (int j = 0; j < 12; ++j) w[i] += M[144 * s + 12 * i + j] * v[12 * s + j];
        }
        for (int i = 0; i < 12; ++i) v[12 * s + i] = w[i];
    }
}

static void mr_blocks_eo(const geom_t *g, double kappa, const cplx *U, const cplx *clov, const cplx *Ainv,
                         int colour, int nmr, const cplx *r, cplx *d, const int32_t *blk, long nblk)
{
    long n = 12 * g->V;
    if (n <= 0) return;
    cplx *rhs = calloc(n, sizeof(cplx)), *rho = calloc(n, sizeof(cplx)), *p = calloc(n, sizeof(cplx));
    cplx *t = calloc(n, sizeof(cplx)), *u = calloc(n, sizeof(cplx)), *w = calloc(n, sizeof(cplx));
    cplx *num = calloc(nblk, sizeof(cplx));
    double *den = calloc(nblk, sizeof(double));

    /* w = A_oo^-1 r_o, t = -kappa H_eo w (in-block), rhs_e = r_e - t */
    for (long i = 0; i < n; ++i) w[i] = r[i];
    if (clov) site_mul(g, Ainv, w, colour, 1);
    wilson_generic(g, kappa, U, NULL, w, t, 0, HOPS_IN_BLOCK, colour, -1, 0, 1);
    for (long s = 0; s < g->V; ++s) {
        int x[4];
        coords(g, s, x);
        int on = colour_of(g, x) == colour && parity_of(x) == 0;
        for (int a = 0; a < 12; ++a) {
            rhs[12 * s + a] = on ? r[12 * s + a] - t[12 * s + a] : 0;
            rho[12 * s + a] = rhs[12 * s + a];
            d[12 * s + a] = 0;
        }
    }
    for (int k = 0; k < nmr; ++k) {
        /* p = A_ee rho - kappa^2 H_eo A_oo^-1 H_oe rho (in-block) */
        wilson_generic(g, kappa, U, NULL, rho, t, 0, HOPS_IN_BLOCK, colour, -1, 1, 0);
        if (clov) site_mul(g, Ainv, t, colour, 1);
        wilson_generic(g, kappa, U, NULL, t, u, 0, HOPS_IN_BLOCK, colour, -1, 0, 1);
        for (long i = 0; i < n; ++i) p[i] = rho[i] - u[i];
        if (clov)  /* + T rho on the even sites of the colour (rho vanishes elsewhere) */
            for (long s = 0; s < g->V; ++s)
                for (int i = 0; i < 12; ++i)
                    for (int j = 0; j < 12; ++j) p[12 * s + i] += clov[144 * s + 12 * i + j] * rho[12 * s + j];
        for (long b = 0; b < nblk; ++b) num[b] = 0, den[b] = 0;
        for (long s = 0; s < g->V; ++s)
            for (int a = 0; a < 12; ++a) {
                num[blk[s]] += conj(p[12 * s + a]) * rho[12 * s + a];
                den[blk[s]] += creal(conj(p[12 * s + a]) * p[12 * s + a]);
            }
        for (long s = 0; s < g->V; ++s) {
            cplx alpha = den[blk[s]] > 0 ? num[blk[s]] / den[blk[s]] : 0;
            for (int a = 0; a < 12; ++a) {
                d[12 * s + a] += alpha * rho[12 * s + a];
                rho[12 * s + a] -= alpha * p[12 * s + a];
            }
        }
    }
    /* d_o = A_oo^-1 (r_o + kappa H_oe d_e) = A_oo^-1 (r_o - t), t = -kappa H_oe d_e (in-block) */
    wilson_generic(g, kappa, U, NULL, d, t, 0, HOPS_IN_BLOCK, colour, -1, 1, 0);
    for (long s = 0; s < g->V; ++s) {
        int x[4];
        coords(g, s, x);
        if (colour_of(g, x) == colour && parity_of(x) == 1)
            for (int a = 0; a < 12; ++a) d[12 * s + a] = r[12 * s + a] - t[12 * s + a];
    }
    if (clov) site_mul(g, Ainv, d, colour, 1);
    free(w);
    free(rhs);
    free(rho);
    free(p);
    free(t);
    free(u);
    free(num);
    free(den);
}

void oracle_sap(const int *L, const int *B, const int *bc, double kappa, const double *Ud, const double *clovd,
                int ncy, int nmr, const double *etad, double *xd)
{
    geom_t g = make_geom(L, B, bc);
    const cplx *U = (const cplx *)Ud;
    const cplx *clov = (const cplx *)clovd;
    cplx *Ainv = clov ? clover_inverse(&g, clov) : NULL;
    const cplx *eta = (const cplx *)etad;
    cplx *x = (cplx *)xd;
    long n = 12 * g.V;
    long nblk = 1;
    for (int mu = 0; mu < 4; ++mu) nblk *= g.L[mu] / g.B[mu];
    int32_t *blk = malloc(g.V * sizeof(int32_t));
    int32_t *col = malloc(g.V * sizeof(int32_t));
    for (long s = 0; s < g.V; ++s) {
        int c[4];
        coords(&g, s, c);
        blk[s] = (int32_t)block_lex(&g, c);
        col[s] = colour_of(&g, c);
    }
    cplx *Dx = malloc(n * sizeof(cplx)), *r = malloc(n * sizeof(cplx)), *d = malloc(n * sizeof(cplx));
    for (long i = 0; i < n; ++i) x[i] = 0;
    for (int cy = 0; cy < ncy; ++cy)
        for (int c = 0; c < 2; ++c) {
            wilson_generic(&g, kappa, U, clov, x, Dx, 1, HOPS_ALL, -1, -1, -1, -1);
            for (long s = 0; s < g.V; ++s)
                for (int a = 0; a < 12; ++a) r[12 * s + a] = col[s] == c ? eta[12 * s + a] - Dx[12 * s + a] : 0;
            mr_blocks_eo(&g, kappa, U, clov, Ainv, c, nmr, r, d, blk, nblk);
            for (long i = 0; i < n; ++i) x[i] += d[i];
        }
    free(blk);
    free(col);
    free(Dx);
    free(r);
    free(d);
    free(Ainv);
}

/* ------------------------------------------------------------------ */
/* Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11).  One round:
 *   (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2   (128-bit products)
 *   c' = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
 * and between rounds the key is bumped by the Weyl constants. */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void oracle_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, c[0], &hi0, &lo0);
        mulhilo64(M1, c[2], &hi1, &lo1);
        uint64_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    for (int i = 0; i < 4; ++i) out[i] = c[i];
}

/*
 * Noise on the canonical lattice.  For site x (canonical index), path step
 * i and noise index k, the words w[4j..4j+3] = Philox(counter = (x, i, k, j),
 * key = (seed, 3)), j = 0..5.
 *   kind 1 (complex Gaussian, E|eta_a|^2 = 1):
 *       u = ((w >> 11) + 1/2) 2^-53;  eta_a = sqrt(-ln u_{2a}) exp(2 pi i u_{2a+1})
 *   kind 0 (Z2): eta_a = 1 - 2 * bit a of w[0]  (real)
 * Sites with mask[x] == 0 (mask may be NULL: all sites) get zero.
 */
void oracle_noise(const int *L, int kind, uint64_t seed, int32_t step, int32_t k, const uint8_t *mask, double *out)
{
    long V = (long)L[0] * L[1] * L[2] * L[3];
    cplx *eta = (cplx *)out;
#pragma omp parallel for schedule(static) if (V >= OMP_MIN_SITES)
    for (long s = 0; s < V; ++s) {
        if (mask && !mask[s]) {
            for (int a = 0; a < 12; ++a) eta[12 * s + a] = 0;
            continue;
        }
        uint64_t key[2] = {seed, 3};
        uint64_t w[24];
        for (int j = 0; j < 6; ++j) {
            uint64_t ctr[4] = {(uint64_t)s, (uint64_t)(uint32_t)step, (uint64_t)(uint32_t)k, (uint64_t)j};
            oracle_philox4x64_10(ctr, key, w + 4 * j);
            if (kind == 0) break;
        }
        for (int a = 0; a < 12; ++a) {
            if (kind == 0) {
                eta[12 * s + a] = 1.0 - 2.0 * (double)((w[0] >> a) & 1);
            } else {
                double u1 = ((double)(w[2 * a] >> 11) + 0.5) * 0x1p-53;
                double u2 = ((double)(w[2 * a + 1] >> 11) + 0.5) * 0x1p-53;
                double rad = sqrt(-log(u1));
                double ph = 2.0 * M_PI * u2;
                eta[12 * s + a] = rad * cos(ph) + I * rad * sin(ph);
            }
        }
    }
}
