/*
 * O2: matrix-free FP64 oracle for the coarse Dirac operator (TEST
 * INFRASTRUCTURE ONLY: called from the test-suite, the smoke check and the
 * CPU baseline of the benchmark; never linked into the product library).
 *
 * Plain C99 + OpenMP, written for checking by eye, not for speed:
 *
 *   D psi(x) = (4 + m0) psi(x)
 *              - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x + mu)
 *                            + (1 + g_mu) U_mu(x - mu)^dag psi(x - mu) ]
 *
 * with the gamma matrices applied as full 4x4 spin matrices (no projection
 * tricks) in the DeGrand-Rossi basis, and a boundary sign bc[mu] on every hop
 * that wraps around direction mu (antiperiodic t: bc[3] = -1).  The paper
 * (section 2) names the Wilson-Dirac operator without writing it; this is the
 * standard r = 1 form.
 *
 * The coarse operator S_bb = D_bb - D_br D_rr^{-1} D_rb (section 1) is applied
 * as  S x = [ D (u - z) ]_b  with u = x scattered to the coarse sites and
 * z = D_rr^{-1} (D u)_r, where D_rr^{-1} is a restarted GCR (Eisenstat, Elman
 * and Schultz 1983; modified Gram-Schmidt, zero initial guess).  The paper's
 * own experiments used BiCGstab (section 4); any convergent solver gives the
 * same S x up to its tolerance.
 *
 * Layout: canonical.  Site s = x + Lx (y + Ly (z + Lz t)); a field is 12
 * complex per site, dof = 12 s + 3 spin + colour; links U[s][mu][row][col].
 * Complex numbers are C99 double complex (interleaved re, im).
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* DeGrand-Rossi gamma matrices, G[mu][row][col], mu = x, y, z, t. */
static cplx G[4][4][4];
static int g_ready = 0;

static void init_gamma(void)
{
    if (g_ready) return;
    memset(G, 0, sizeof G);
    /* gamma_x */
    G[0][0][3] = I;  G[0][1][2] = I;  G[0][2][1] = -I; G[0][3][0] = -I;
    /* gamma_y */
    G[1][0][3] = -1; G[1][1][2] = 1;  G[1][2][1] = 1;  G[1][3][0] = -1;
    /* gamma_z */
    G[2][0][2] = I;  G[2][1][3] = -I; G[2][2][0] = -I; G[2][3][1] = I;
    /* gamma_t */
    G[3][0][2] = 1;  G[3][1][3] = 1;  G[3][2][0] = 1;  G[3][3][1] = 1;
    g_ready = 1;
}

typedef struct {
    long L[4];
    int bc[4];
    long V;
    const cplx *U; /* [V][4][3][3] */
    double m0;
} op_t;

static void op_init(op_t *op, const int32_t dims[4], const int32_t bc[4],
                    const double *links, double m0)
{
    init_gamma();
    op->V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        op->L[mu] = dims[mu];
        op->bc[mu] = bc[mu];
        op->V *= dims[mu];
    }
    op->U = (const cplx *)links;
    op->m0 = m0;
}

/* neighbour of s one step (+1 / -1) along mu, with the wrap sign */
static long neighbour(const op_t *op, long s, int mu, int step, double *sign)
{
    long c[4], r = s;
    for (int nu = 0; nu < 4; ++nu) {
        c[nu] = r % op->L[nu];
        r /= op->L[nu];
    }
    long n = c[mu] + step;
    *sign = 1.0;
    if (n < 0 || n >= op->L[mu]) {
        *sign = (double)op->bc[mu];
        n = (n + op->L[mu]) % op->L[mu];
    }
    c[mu] = n;
    return c[0] + op->L[0] * (c[1] + op->L[1] * (c[2] + op->L[2] * c[3]));
}

static const cplx *link(const op_t *op, long s, int mu)
{
    return op->U + 9 * (4 * s + mu);
}

/*
 * out = mask_out D mask_in (in):  rows restricted to sites with
 * omask[s] == osel, columns to sites with imask[s] == isel.  A NULL mask
 * selects every site.  Rows outside the selection are set to zero.
 */
static void apply_block(const op_t *op, const unsigned char *omask, int osel,
                        const unsigned char *imask, int isel,
                        const cplx *in, cplx *out)
{
    const long V = op->V;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        cplx acc[12];
        if (omask && omask[s] != osel) {
            for (int k = 0; k < 12; ++k) out[12 * s + k] = 0;
            continue;
        }
        for (int k = 0; k < 12; ++k)
            acc[k] = (!imask || imask[s] == isel) ? (4.0 + op->m0) * in[12 * s + k] : 0;
        for (int mu = 0; mu < 4; ++mu) {
            for (int dir = 0; dir < 2; ++dir) {
                double sign;
                long n = neighbour(op, s, mu, dir == 0 ? +1 : -1, &sign);
                if (imask && imask[n] != isel) continue;
                /* chi[spin][a] = W psi(n)[spin][.], W = U_mu(s) or U_mu(s-mu)^dag */
                const cplx *u = dir == 0 ? link(op, s, mu) : link(op, n, mu);
                cplx chi[4][3];
                for (int sp = 0; sp < 4; ++sp)
                    for (int a = 0; a < 3; ++a) {
                        cplx t = 0;
                        for (int b = 0; b < 3; ++b) {
                            cplx w = dir == 0 ? u[3 * a + b] : conj(u[3 * b + a]);
                            t += w * in[12 * n + 3 * sp + b];
                        }
                        chi[sp][a] = t;
                    }
                /* acc -= 1/2 sign (1 -/+ gamma_mu) chi */
                double pm = dir == 0 ? -1.0 : +1.0;
                for (int i = 0; i < 4; ++i)
                    for (int a = 0; a < 3; ++a) {
                        cplx t = 0;
                        for (int j = 0; j < 4; ++j) {
                            cplx p = (i == j ? 1.0 : 0.0) + pm * G[mu][i][j];
                            t += p * chi[j][a];
                        }
                        acc[3 * i + a] -= 0.5 * sign * t;
                    }
            }
        }
        for (int k = 0; k < 12; ++k) out[12 * s + k] = acc[k];
    }
}

/*
 * The sum of the absolute values of the terms that make up each output of
 * apply_block: every product of a spin-matrix entry, a link entry and an
 * input entry, taken in absolute value (|1 -/+ gamma| entries, |U| entries,
 * |psi| entries), plus |4 + m0| |psi(x)| when diag != 0.  For lattices with
 * every extent >= 3 no two hops join the same pair of sites, so this is
 * |D| |psi| with |D| the entrywise absolute value of the matrix.  It scales
 * the rounding error of any evaluation of the sum: an evaluation whose
 * inputs carry a relative error e has an output error of at most
 * e times this value.  Real output, [nrhs][12 V].
 */
static void apply_block_abs(const op_t *op, const unsigned char *omask, int osel,
                            const unsigned char *imask, int isel, int diag,
                            const cplx *in, double *out)
{
    const long V = op->V;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        double acc[12];
        if (omask && omask[s] != osel) {
            for (int k = 0; k < 12; ++k) out[12 * s + k] = 0;
            continue;
        }
        for (int k = 0; k < 12; ++k)
            acc[k] = (diag && (!imask || imask[s] == isel)) ? fabs(4.0 + op->m0) * cabs(in[12 * s + k]) : 0;
        for (int mu = 0; mu < 4; ++mu) {
            for (int dir = 0; dir < 2; ++dir) {
                double sign;
                long n = neighbour(op, s, mu, dir == 0 ? +1 : -1, &sign);
                if (imask && imask[n] != isel) continue;
                const cplx *u = dir == 0 ? link(op, s, mu) : link(op, n, mu);
                double pm = dir == 0 ? -1.0 : +1.0;
                for (int i = 0; i < 4; ++i)
                    for (int a = 0; a < 3; ++a)
                        for (int j = 0; j < 4; ++j) {
                            double p = cabs((i == j ? 1.0 : 0.0) + pm * G[mu][i][j]);
                            if (p == 0) continue;
                            for (int b = 0; b < 3; ++b) {
                                cplx w = dir == 0 ? u[3 * a + b] : conj(u[3 * b + a]);
                                acc[3 * i + a] += 0.5 * p * cabs(w) * cabs(in[12 * n + 3 * j + b]);
                            }
                        }
            }
        }
        for (int k = 0; k < 12; ++k) out[12 * s + k] = acc[k];
    }
}

/* ------------------------------------------------------------ vector ops */
static cplx vdot(long n, const cplx *a, const cplx *b) /* sum conj(a) b */
{
    double re = 0, im = 0;
#pragma omp parallel for schedule(static) reduction(+ : re, im)
    for (long i = 0; i < n; ++i) {
        cplx t = conj(a[i]) * b[i];
        re += creal(t);
        im += cimag(t);
    }
    return re + I * im;
}

static double vnorm(long n, const cplx *a) { return sqrt(creal(vdot(n, a, a))); }

static void vaxpy(long n, cplx alpha, const cplx *x, cplx *y) /* y += alpha x */
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) y[i] += alpha * x[i];
}

static void vscale(long n, cplx alpha, cplx *x)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) x[i] *= alpha;
}

static void vcopy(long n, const cplx *x, cplx *y)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) y[i] = x[i];
}

/* ------------------------------------------------------------ GCR for D_rr */
typedef struct {
    const op_t *op;
    const unsigned char *mask; /* 1 on coarse (b) sites, 0 on the rest (r) */
} drr_t;

static void drr_apply(const drr_t *A, const cplx *in, cplx *out)
{
    apply_block(A->op, A->mask, 0, A->mask, 0, in, out);
}

/*
 * Restarted GCR(m) for D_rr x = b, zero initial guess, right preconditioner
 * M = 1.  Vectors live on the full lattice and vanish on coarse sites.
 * Returns the iteration count; *relres receives the true residual
 * ||b - D_rr x|| / ||b|| recomputed at exit.
 */
static int gcr_drr(const drr_t *A, const cplx *b, cplx *x, int m, double tol,
                   int maxit, double *relres)
{
    const long n = 12 * A->op->V;
    cplx *r = malloc(sizeof(cplx) * n);
    cplx *P = malloc(sizeof(cplx) * n * m);
    cplx *Q = malloc(sizeof(cplx) * n * m);
    memset(x, 0, sizeof(cplx) * n);
    vcopy(n, b, r);
    const double bnorm = vnorm(n, b);
    int it = 0, k = 0;
    if (bnorm == 0.0) {
        *relres = 0.0;
        free(r); free(P); free(Q);
        return 0;
    }
    while (it < maxit) {
        cplx *p = P + n * k, *q = Q + n * k;
        vcopy(n, r, p);          /* p = M r with M = 1 */
        drr_apply(A, p, q);      /* q = A p */
        for (int j = 0; j < k; ++j) {
            cplx beta = vdot(n, Q + n * j, q);
            vaxpy(n, -beta, Q + n * j, q);
            vaxpy(n, -beta, P + n * j, p);
        }
        double nu = vnorm(n, q);
        vscale(n, 1.0 / nu, q);
        vscale(n, 1.0 / nu, p);
        cplx alpha = vdot(n, q, r);
        vaxpy(n, alpha, p, x);
        vaxpy(n, -alpha, q, r);
        ++it;
        if (vnorm(n, r) <= tol * bnorm) break;
        if (++k == m) {          /* restart from the true residual */
            k = 0;
            drr_apply(A, x, r);
            for (long i = 0; i < n; ++i) r[i] = b[i] - r[i];
        }
    }
    drr_apply(A, x, r);
    for (long i = 0; i < n; ++i) r[i] = b[i] - r[i];
    *relres = vnorm(n, r) / bnorm;
    free(r); free(P); free(Q);
    return it;
}

static unsigned char *coarse_mask(long V, const int32_t *q, int32_t nb)
{
    unsigned char *mask = calloc((size_t)V, 1);
    for (int32_t k = 0; k < nb; ++k) mask[q[k]] = 1;
    return mask;
}

/* ------------------------------------------------------------ exported API */
int orc_num_threads(void) { return omp_get_max_threads(); }

/* out = D in for nrhs fields (canonical layout). */
int orc_dirac_apply(const int32_t dims[4], const int32_t bc[4], const double *links,
                    double m0, const double *in, double *out, int nrhs)
{
    op_t op;
    op_init(&op, dims, bc, links, m0);
    for (int k = 0; k < nrhs; ++k)
        apply_block(&op, NULL, 0, NULL, 0, (const cplx *)in + 12 * op.V * k,
                    (cplx *)out + 12 * op.V * k);
    return 0;
}

/* out = mask_osel D mask_isel in; sel = 1 selects coarse sites q[0:nb]. */
int orc_block_apply(const int32_t dims[4], const int32_t bc[4], const double *links,
                    double m0, const int32_t *q, int32_t nb, int osel, int isel,
                    const double *in, double *out, int nrhs)
{
    op_t op;
    op_init(&op, dims, bc, links, m0);
    unsigned char *mask = coarse_mask(op.V, q, nb);
    for (int k = 0; k < nrhs; ++k)
        apply_block(&op, mask, osel, mask, isel, (const cplx *)in + 12 * op.V * k,
                    (cplx *)out + 12 * op.V * k);
    free(mask);
    return 0;
}

/* out = the absolute-value sums of mask_osel D mask_isel in (real [nrhs][12 V]);
 * diag = 0 leaves out the diagonal term (the hopping part alone). */
int orc_block_apply_abs(const int32_t dims[4], const int32_t bc[4], const double *links,
                        double m0, const int32_t *q, int32_t nb, int osel, int isel, int diag,
                        const double *in, double *out, int nrhs)
{
    op_t op;
    op_init(&op, dims, bc, links, m0);
    unsigned char *mask = coarse_mask(op.V, q, nb);
    for (int k = 0; k < nrhs; ++k)
        apply_block_abs(&op, mask, osel, mask, isel, diag, (const cplx *)in + 12 * op.V * k,
                        out + 12 * op.V * k);
    free(mask);
    return 0;
}

/* D_rr x = b for nrhs right-hand sides (full-lattice layout, zero on b). */
int orc_drr_solve(const int32_t dims[4], const int32_t bc[4], const double *links,
                  double m0, const int32_t *q, int32_t nb, const double *b, double *x,
                  int nrhs, int restart, double tol, int maxit, int32_t *iters,
                  double *relres)
{
    op_t op;
    op_init(&op, dims, bc, links, m0);
    unsigned char *mask = coarse_mask(op.V, q, nb);
    drr_t A = {&op, mask};
    int status = 0;
    for (int k = 0; k < nrhs; ++k) {
        iters[k] = gcr_drr(&A, (const cplx *)b + 12 * op.V * k,
                           (cplx *)x + 12 * op.V * k, restart, tol, maxit, &relres[k]);
        if (!(relres[k] <= tol)) status = 1;
    }
    free(mask);
    return status;
}

/* ||b - D_rr x|| / ||b|| per right-hand side. */
int orc_drr_residual(const int32_t dims[4], const int32_t bc[4], const double *links,
                     double m0, const int32_t *q, int32_t nb, const double *b,
                     const double *x, int nrhs, double *relres)
{
    op_t op;
    op_init(&op, dims, bc, links, m0);
    unsigned char *mask = coarse_mask(op.V, q, nb);
    drr_t A = {&op, mask};
    const long n = 12 * op.V;
    cplx *r = malloc(sizeof(cplx) * n);
    for (int k = 0; k < nrhs; ++k) {
        const cplx *bk = (const cplx *)b + n * k;
        drr_apply(&A, (const cplx *)x + n * k, r);
        for (long i = 0; i < n; ++i) r[i] = bk[i] - r[i];
        double bn = vnorm(n, bk);
        relres[k] = bn > 0 ? vnorm(n, r) / bn : vnorm(n, r);
    }
    free(r);
    free(mask);
    return 0;
}

/*
 * y_b = S_bb x_b for nrhs coarse vectors ([nrhs][12 nb], coarse index k is
 * site q[k]).  iters/relres receive the D_rr solve statistics per RHS.
 */
int orc_schur_apply(const int32_t dims[4], const int32_t bc[4], const double *links,
                    double m0, const int32_t *q, int32_t nb, const double *xb,
                    double *yb, int nrhs, int restart, double tol, int maxit,
                    int32_t *iters, double *relres)
{
    op_t op;
    op_init(&op, dims, bc, links, m0);
    unsigned char *mask = coarse_mask(op.V, q, nb);
    drr_t A = {&op, mask};
    const long n = 12 * op.V;
    cplx *u = malloc(sizeof(cplx) * n), *y = malloc(sizeof(cplx) * n);
    cplx *z = malloc(sizeof(cplx) * n), *w = malloc(sizeof(cplx) * n);
    int status = 0;
    for (int k = 0; k < nrhs; ++k) {
        const cplx *x = (const cplx *)xb + 12L * nb * k;
        cplx *out = (cplx *)yb + 12L * nb * k;
        memset(u, 0, sizeof(cplx) * n);
        for (int32_t j = 0; j < nb; ++j)
            for (int d = 0; d < 12; ++d) u[12L * q[j] + d] = x[12L * j + d];
        apply_block(&op, mask, 0, mask, 1, u, y);     /* y = D_rb x */
        iters[k] = gcr_drr(&A, y, z, restart, tol, maxit, &relres[k]);
        if (!(relres[k] <= tol)) status = 1;
        for (long i = 0; i < n; ++i) u[i] -= z[i];      /* u - z */
        apply_block(&op, mask, 1, NULL, 0, u, w);        /* [D (u - z)]_b */
        for (int32_t j = 0; j < nb; ++j)
            for (int d = 0; d < 12; ++d) out[12L * j + d] = w[12L * q[j] + d];
    }
    free(u); free(y); free(z); free(w);
    free(mask);
    return status;
}
