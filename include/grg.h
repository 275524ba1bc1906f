/*
 * grg.h -- C ABI of the MI355X (gfx950) library for the coarse Dirac operator
 * of a one-step gauged renormalisation-group blocking of Wilson fermions
 * (A. Borici, "On Gauged Renormalisation Group Transformations of Lattice
 * Fermions", arXiv:0704.2341).
 *
 * The operator.  After a site permutation that labels the coarse sites first,
 * the Wilson-Dirac matrix is partitioned as D = [[D_bb, D_br], [D_rb, D_rr]]
 * (section 1, step 1) and the coarse operator is the Schur complement
 *     S_bb = D_bb - D_br D_rr^{-1} D_rb                 (section 1)
 * of the block-UL factorisation.  Applying S_bb needs a solve with D_rr
 * (section 2, closing remark on cost), which dominates the run time.
 *
 * The Wilson operator (the paper names it without writing it out; the
 * standard r = 1 form in the DeGrand-Rossi basis):
 *     D psi(x) = (4 + m0) psi(x)
 *       - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu) ]
 * with a sign bc[mu] (+1 periodic, -1 antiperiodic) on hops that wrap.
 *
 * Layout at the boundary (canonical; the internal layout is private):
 *   - dims = {Lx, Ly, Lz, Lt}; site s = x + Lx (y + Ly (z + Lz t)), x fastest;
 *   - a lattice field is 12 complex128 per site, dof = 12 s + 3 spin + colour,
 *     interleaved (re, im) doubles; a batch of nrhs fields is [nrhs][12 V];
 *   - links are [V][4][3][3] complex128, U[s][mu][row][col], mu = x, y, z, t;
 *   - a coarse-space field is [nrhs][12 N_b] complex128; coarse index k is
 *     lattice site q[k] of the ordering vector (see grg_permutation_block).
 *
 * Ownership and memory: field and link pointers passed to the compute calls
 * are DEVICE pointers owned by the caller (e.g. torch tensors); the library
 * never frees them.  Handles and every workspace are owned by the library:
 * workspaces are allocated by *_create for a stated maximum nrhs, so the
 * apply/solve calls do not allocate.  Work is enqueued on the stream given at
 * lattice creation; every call returns after that stream has drained.
 * Handles must not be used from two threads at once.
 *
 * Errors: every call returns a grg_status and never aborts or throws across
 * the boundary.  Arguments are validated before anything is enqueued.  The
 * message of the last failure in the calling thread is grg_last_error().
 * Every apply and solve call takes nrhs in 1..max_rhs of its handle (1..16
 * for the lattice calls): an empty batch, nrhs = 0, is GRG_EINVAL and writes
 * nothing.
 */
#ifndef GRG_H
#define GRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GRG_OK = 0,
    GRG_EINVAL = -1,       /* invalid argument (null pointer, bad size, ...) */
    GRG_EODD_EXTENT = -2,  /* Type I/II blocking needs even extents */
    GRG_ENOMEM = -3,       /* device or host allocation failed */
    GRG_EHIP = -4,         /* HIP runtime error; text in grg_last_error() */
    GRG_ENOCONV = -5,      /* solver hit its iteration cap; best iterate returned */
    GRG_ENONFINITE = -6,   /* NaN or Inf met in a residual */
    GRG_ETOO_LARGE = -7,   /* output would exceed the caller's capacity */
    GRG_EUNSUPPORTED = -8  /* valid request that this library does not support */
} grg_status;

typedef enum { GRG_PERM_I = 1, GRG_PERM_II = 2 } grg_perm_type;

/* Storage/arithmetic of a dslash or of the inner solve.  GRG_BF16 stores
 * fields and links in bfloat16 and computes in FP32. */
typedef enum { GRG_FP64 = 0, GRG_FP32 = 1, GRG_BF16 = 2 } grg_precision;

typedef struct grg_lattice_s *grg_lattice;
typedef struct grg_schur_s *grg_schur;
typedef struct grg_precond_s *grg_precond;

/* Parameters of the D_rr solve.  Restarted GCR(restart) with the residual
 * carried through restarts (restart = 1 is minimal residual).  With
 * inner = GRG_FP64 the whole solve is FP64; otherwise an FP64 defect
 * correction wraps inner solves in the given precision, each reducing its
 * residual by inner_tol. */
typedef struct {
    double tol;        /* target: ||b - D_rr x|| <= tol ||b|| in FP64, per RHS */
    int max_iter;      /* cap on inner iterations per solve (summed over outer) */
    int restart;       /* GCR restart length m >= 1 */
    int inner;         /* grg_precision of the inner iterations */
    double inner_tol;  /* relative reduction per inner solve (mixed only) */
    int max_outer;     /* cap on defect-correction steps (mixed only) */
    int max_rhs;       /* largest nrhs per call; sizes the workspaces (<= 16) */
    int check_every;   /* iterations between host-side convergence checks */
    int verify;        /* 1: on convergence, recompute b - D_rr x from x in FP64 and resume
                          if it misses tol; 0 (default): stop on the defect correction's
                          FP64 residual, which is updated with the exact FP64 operator
                          and equals b - D_rr x up to FP64 rounding */
    int eo;            /* 1 (default): inner solves with restart 1 (minimal residual, its
                          flexible form with the learned preconditioner) and BiCGstab run on
                          the even-odd reduced system of D_rr when every extent is even and
                          d = 4 + m0 is not zero (the
                          hopping term couples opposite parities: solve
                          (d - H_pq H_qp / d) z_p = b_p - H_pq b_q / d on one parity, then
                          z_q = (b_q - H_qp z_p) / d); 0: on D_rr itself */
    int method;        /* 0 (default): GCR(restart) as above; 1: BiCGstab (van der Vorst's
                          stabilised biconjugate gradients, the D_rr solver of the paper's
                          section 4 experiment: two operator applications per iteration,
                          shadow residual = the initial residual); ignores restart and the
                          learned preconditioner */
} grg_solver_params;

typedef struct {
    int iters;             /* inner iterations taken (all outer steps) */
    int outer;             /* defect-correction steps (0 for plain FP64) */
    int converged;         /* 1 if every RHS met tol */
    int n_dslash;          /* dslash launches in the call */
    double true_rel_resid; /* max over RHS of the FP64 ||b - D_rr x|| / ||b|| */
    double t_total_ms;     /* wall time of the call on the stream */
    double t_dslash_ms;    /* summed stencil time: D_rr, D_rb and the reduced operator's
                              half-lattice stencils (only with profiling on; this and
                              the other phase times are -1 with launch-only
                              profiling) */
    int fallbacks;         /* inner solves redone without the preconditioner */
    double t_dc_ms;        /* summed time of the FP64 defect-correction steps (stencil and
                              residual update fused; profiling on) */
    double t_blas_ms;      /* summed time of the Krylov vector kernels: updates, norms,
                              reductions, conversions, the final sum of the corrections
                              (profiling on) */
    double t_prec_ms;      /* summed time of the learned preconditioner's applications
                              inside the solve (profiling on) */
} grg_solver_stats;

/* Training of the learned preconditioner (see grg_precond_train). */
typedef struct {
    int steps;          /* optimiser steps */
    int batch;          /* residual/error pairs per step (<= the schur's max_rhs) */
    int max_mr_steps;   /* pairs come from 0..max_mr_steps minimal-residual steps */
    double lr;          /* Adam learning rate (beta1 0.9, beta2 0.999, eps 1e-8) */
    uint64_t seed;      /* seeds the random errors and the step counts */
    int log_every;      /* loss read back every log_every steps (0: first/last only) */
    int reduced;        /* 1: after a first quarter of the steps on pairs of D_rr itself, pairs
                           of the even-odd reduced D_rr system (inputs, errors and the loss
                           on the reduced parity's rest sites), for the reduced inner solve
                           that uses the network restricted to that parity; needs even
                           extents.  (On pairs of one parity alone the hop weights get no
                           gradient while they are zero, as at the identity start.)
                           0: pairs of D_rr itself */
} grg_train_params;

typedef struct {
    int steps;
    int pairs;          /* residual/error pairs consumed */
    double loss_first;  /* loss of the first minibatch */
    double loss_last;   /* mean loss of the last log_every minibatches */
    double t_ms;
} grg_train_stats;

/* Thread-local message of the last failure; never NULL. */
const char *grg_last_error(void);
const char *grg_version(void);

/* Fill p with the defaults (tol 1e-10, restart 1, FP64, max_rhs 12, ...). */
grg_status grg_solver_params_default(grg_solver_params *p);

/* Lattice geometry and the stream all work of this lattice runs on.
 * dims: four positive extents; bc: +1 / -1 per direction; stream: a
 * hipStream_t (NULL = default stream).  The current HIP device is recorded. */
grg_status grg_lattice_create(const int32_t dims[4], const int32_t bc[4], void *stream,
                              grg_lattice *out);
grg_status grg_lattice_destroy(grg_lattice lat);
grg_status grg_lattice_volume(grg_lattice lat, int64_t *volume);

/* Set the gauge field from canonical links (host pointer if on_device == 0,
 * device pointer otherwise).  Copies are made in every precision.  Schur
 * handles and learned preconditioners on lat read the links at every call,
 * so they follow a new field from their next call; a V-cycle hierarchy
 * blocks the links into its coarse lattices when it is created and must be
 * created again after the field changes.  Must not overlap a call that uses
 * lat. */
grg_status grg_gauge_set(grg_lattice lat, const double *links, int on_device);

/* The site permutation of section 2 (Permutation_block): q[k] is the site
 * placed at row k, coarse sites first.  Type I blocks in all directions at
 * once (coarse = all-even sites); Type II blocks one direction at a time
 * (nested red-black, x first).  inverse != 0 returns the inverse ordering
 * (operator P^T).  q: host array of V int32, caller-owned.  *n_coarse = V/16.
 * Odd extents give GRG_EODD_EXTENT.  Host-only: no device work. */
grg_status grg_permutation_block(const int32_t dims[4], int type, int inverse, int32_t *q,
                                 int32_t *n_coarse);

/* out = D in for nrhs canonical lattice fields (device pointers): the
 * Wilson-Dirac operator written out at the top of this header, the fine
 * operator D that section 1 partitions and whose spectrum section 2's
 * Figure 2 shows before and after blocking.  Computed in the given precision:
 * inputs and links are rounded to it (BF16 through FP32, round to nearest
 * even), the arithmetic is FP64, FP32 or FP32 on BF16 operands, and the result
 * is widened to FP64.  Uses a grow-only scratch of the lattice handle (two
 * fields of nrhs in that precision, allocated on the first call that needs
 * more).  GRG_EINVAL: null pointer, nrhs outside 1..16, bad precision, gauge
 * field not set, m0 not finite. */
grg_status grg_dirac_apply(grg_lattice lat, double m0, int precision, const double *in,
                           double *out, int nrhs);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): out = D in
 * exactly as grg_dirac_apply (same kernels and launch, so the same bits), but
 * its two internal staging fields live in a fixed scratch array of
 * GRG_NOALLOC_SCRATCH_BYTES per GPU that the library holds until the process
 * ends, so the call itself allocates nothing (the first call on a device
 * looks up that device's array once).  Needs
 *     2 * ceil256(12 * Vs * nrhs * b) <= GRG_NOALLOC_SCRATCH_BYTES,
 * b = 16, 8, 4 bytes for FP64, FP32, BF16 and Vs = V rounded up to a multiple
 * of 256 (e.g. 8^4 with 16 RHS in FP64, 16^4 with 1 RHS); larger requests
 * return GRG_ETOO_LARGE before anything is enqueued.  Other errors as
 * grg_dirac_apply.  Every call on one GPU uses that GPU's one array: calls
 * that overlap in time on one GPU (two threads, or two streams without
 * ordering) race and give wrong results; calls ordered on one stream are
 * safe.  No entry of the array is read before the call writes it. */
#define GRG_NOALLOC_SCRATCH_BYTES (32u << 20)
grg_status grg_dirac_apply_noalloc(grg_lattice lat, double m0, int precision, const double *in,
                                   double *out, int nrhs);

/* The coarse operator S_bb = D_bb - D_br D_rr^{-1} D_rb (section 1) of the
 * partition of D induced by the ordering q: section 1, step 1 splits D into
 * the 2x2 blocks of the coarse sites (the first n_coarse entries of q) and
 * the rest, with q from section 2's Permutation_block (coarse sites labelled
 * first).  q: host, V entries, a permutation of the sites (checked);
 * n_coarse in 1..V-1.  Allocates every workspace for params->max_rhs
 * right-hand sides (params NULL = defaults), and the inner-precision
 * workspaces on the first solve that needs them.  GRG_EINVAL on a bad q,
 * n_coarse or parameter; GRG_ENOMEM if a workspace cannot be allocated. */
grg_status grg_schur_create(grg_lattice lat, double m0, const int32_t *q, int32_t n_coarse,
                            const grg_solver_params *params, grg_schur *out);
grg_status grg_schur_destroy(grg_schur s);
grg_status grg_schur_set_params(grg_schur s, const grg_solver_params *params);

/* x = D_rr^{-1} rhs for nrhs canonical lattice fields (device): the solve
 * with the rest-site block that S_bb needs (section 1, the S_bb formula), and
 * the cost section 2 points at (computing S_bb requires inverting D_rr).
 * Solved to ||rhs - D_rr x|| <= params.tol ||rhs|| per RHS in FP64 (the
 * defect correction's FP64 residual, see grg_solver_params).  Entries of rhs
 * on coarse sites are ignored; x is zero there.  GRG_ENOCONV (an iteration
 * cap met): per RHS, x is the iterate of smallest FP64 residual among the
 * defect-correction steps (x = 0 included) since the corrections were last
 * summed into the iterate (every 16 steps, so normally the best overall),
 * and stats->true_rel_resid is its residual.  GRG_ENONFINITE on a NaN or Inf
 * residual.  stats may be NULL. */
grg_status grg_drr_solve(grg_schur s, const double *rhs, double *x, int nrhs,
                         grg_solver_stats *stats);

/* y_b = S_bb x_b for nrhs coarse fields [nrhs][12 N_b] (device), the
 * Schur complement of section 1 applied matrix-free:
 * S x = [ D (u - D_rr^{-1} (D u)_r) ]_b with u = x on the coarse sites (the
 * block-UL factorisation of section 1: its lower factor's first block
 * column).  The D_rr solve as grg_drr_solve; errors as grg_drr_solve. */
grg_status grg_schur_apply(grg_schur s, const double *x_b, double *y_b, int nrhs,
                           grg_solver_stats *stats);

/* The dense S_bb, column-major (12 N_b)^2 complex128 in HOST memory
 * (caller-owned), by applying S_bb to unit vectors: what section 2's
 * Schur_complement computes, for the spectra of section 2 (Figure 2) at small
 * volume.  GRG_ETOO_LARGE if (12 N_b)^2 * 16 bytes exceeds cap_bytes. */
grg_status grg_schur_assemble(grg_schur s, double *S, size_t cap_bytes);

/* The second-order Schur complement approximation of section 3,
 *     S~_bb = D_bb - D_br (d^{-1} + d~^{-1} - d^{-1} D_rr d~^{-1}) D_rb,
 * with d the diagonal of D_rr (4 + m0) and d~ the diagonal matrix of the row
 * sums of D_rr, each scalar row summed over its dof (d~ = D_rr applied to the
 * field that is 1 on every rest-site dof).  y_b = S~_bb x_b for nrhs
 * coarse-space fields (device, layout as grg_schur_apply), in FP64: four
 * stencil launches and no solve.  GRG_EINVAL if 4 + m0 = 0; a zero row sum
 * gives non-finite output (no check).  Uses the handle's workspaces. */
grg_status grg_reusken_apply(grg_schur s, const double *x_b, double *y_b, int nrhs);
/* Dense S~_bb (host, column-major complex128), as grg_schur_assemble. */
grg_status grg_reusken_assemble(grg_schur s, double *S, size_t cap_bytes);

/* The approximation that section 3 contrasts with the second-order one:
 * the couplings inside D_rr ignored, which keeps the sparsity pattern of the
 * coarse operator (it couples coarse sites at most two fine hops apart):
 *     S0_bb = D_bb - D_br d^{-1} D_rb,   d = 4 + m0, the diagonal of D_rr.
 * y_b = S0_bb x_b for nrhs coarse-space fields (device, layout as
 * grg_schur_apply), in FP64: two stencil launches, no solve.  GRG_EINVAL if
 * 4 + m0 = 0.  Uses the handle's workspaces. */
grg_status grg_diag_schur_apply(grg_schur s, const double *x_b, double *y_b, int nrhs);
/* The dense S0_bb, as grg_schur_assemble. */
grg_status grg_diag_schur_assemble(grg_schur s, double *S, size_t cap_bytes);

/* Autotuner: time every candidate launch shape of the stencil (sites per
 * workgroup, right-hand sides per thread, hop grouping, grid size) for nrhs
 * right-hand sides, in FP64 and in the inner precision, and of the fused
 * defect-correction step, on this handle's workspaces, and keep the fastest
 * for later calls with that nrhs.  Every candidate evaluates each site in the
 * same order, so tuning changes speed, not results.  Takes a few hundred
 * stencil launches; overwrites the handle's workspaces (not caller memory). */
grg_status grg_schur_tune(grg_schur s, int nrhs);
/* The launch used for (precision, nrhs): info = {sites per workgroup, RHS per
 * thread (site-parallel kernel) or per workgroup (t-marching kernel),
 * hop schedule (0: one direction per loop iteration, 1: one hop per
 * iteration, 2: BF16 only, straight-line with the next hop's loads issued
 * before the current hop's arithmetic), workgroups, items per XCD chunk (0 = one
 * contiguous eighth of the lattice per XCD), time-chunk length of the
 * t-marching kernel (0 = site-parallel kernel)}; *ms = its tuned time per
 * launch, or -1 if untuned (defaults in use).  precision 3..5 reports the
 * half-lattice stencil of the even-odd reduced solve in precision - 3, whose
 * hop schedules 3..6 are BF16 only: 3 is its t-marching form (info[0] =
 * 256), a workgroup holding 64 columns of the half lattice and four RHS,
 * walking info[5] time slices; 4 and 5 carry info[1] = 2 or 3 RHS through
 * each hop together; 6 takes the x hops' spinors from lane shuffles; 7 is
 * the plane form of the t-marching stencil (info[0] = Lx / 2 * Ly, a multiple
 * of 64 and at most 512), a workgroup holding a whole x-y plane of the half
 * lattice for one RHS (info[1] = 1), or two planes z, z + 1 of it (info[1] =
 * 2, Lz a multiple of 16, the z hop between the two from LDS), walking
 * info[5] time slices with the x, y and backward t hops read from LDS;
 * info[5] = 0 except with 3 and 7.  With
 * schedule 3 or 7, the full-layout first and last steps of a reduced solve
 * run the one-hop shape that tuning found faster for them, if it found one,
 * else the same schedule as well. */
grg_status grg_schur_tune_info(grg_schur s, int precision, int nrhs, int32_t info[6], float *ms);

/* Pin the stencil launch for (precision, nrhs), e.g. from a saved tuning
 * result: info as returned by grg_schur_tune_info.  GRG_EINVAL if the shape
 * is not valid for this lattice (a t-marching workgroup holds 64 * RHS
 * threads, at most 512 in FP64 and 768 otherwise; the t-marching
 * half-lattice stencil needs a multiple of 64 half-sites per time slice, its
 * plane form an x-y plane of 64 to 512 half-sites, a multiple of 64). */
grg_status grg_schur_set_launch(grg_schur s, int precision, int nrhs, const int32_t info[6]);

/* The launch of the fused FP64 defect-correction step r -= D_rr e / s,
 * x += e / s (inner solution e stored in `precision`), for nrhs RHS: info as
 * in grg_schur_tune_info, where info[5] = 0 selects the site-parallel kernel
 * (info[0] threads per workgroup: 64, 128 or 256) and info[5] = T > 0 the
 * t-marching kernel (64 * info[1] <= 512 threads, time chunks of T);
 * info[2] = 1 selects the LDS-ring form of the t-marching kernel (BF16 inner
 * precision, Lx dividing 64, a multiple of 64 sites per x-y-z slice and at
 * most 4 RHS per workgroup; the column's e at t - 1 and t and its U_t at
 * t - 1 kept in LDS, each site finished within its slice), 3 the same with
 * the work items ordered RHS group first (the groups
 * of a tile run together on one XCD and share its links), else 0.
 * *ms = tuned time per step, or -1 if untuned. */
grg_status grg_schur_dc_launch_info(grg_schur s, int precision, int nrhs, int32_t info[6],
                                    float *ms);
/* Pin that launch; GRG_EINVAL if the shape is not valid for this lattice. */
grg_status grg_schur_set_dc_launch(grg_schur s, int precision, int nrhs, const int32_t info[6]);

/* The sub-blocks of the partition (section 1, step 1): out = D_{rows,cols} in
 * for nrhs canonical lattice fields (device), with rows / cols = 1 for the
 * coarse sites, 0 for the rest, -1 for every site; in is read only on the
 * cols sites and out is zero off the rows sites.  Computed in the given
 * precision with the handle's stencil launch.  D_rr is the operator the solve
 * inverts; D_rb, D_br and D_bb enter S_bb. */
grg_status grg_block_apply(grg_schur s, int precision, int rows, int cols, const double *in,
                           double *out, int nrhs);

/* The even-odd reduced form of D_rr on one parity: D_rr couples a rest site
 * only to itself (diagonal d = 4 + m0) and to rest sites of the other parity,
 * so on the rest sites of parity p (x + y + z + t mod 2) and q = 1 - p its
 * Schur complement is A_p = d - H_pq H_qp / d, with H the hopping part of
 * D_rr (the same block elimination as S_bb, applied to D_rr; the reduced
 * solve works on it).  out = A_p in for nrhs canonical lattice fields
 * (device); in is read on the rest sites of parity p only and out is zero
 * elsewhere.  Computed in the given precision with the two half-lattice
 * stencils of the handle's launch (grg_schur_tune_info, precision 3..5).
 * GRG_EINVAL if an extent is odd (no even-odd form), 4 + m0 = 0 (no reduced
 * form) or parity is not 0 or 1. */
grg_status grg_reduced_apply(grg_schur s, int precision, int parity, const double *in, double *out,
                             int nrhs);

/* ---------------------------------------------------------------------------
 * Cyclic-reduction V-cycle (section 4): a multilevel preconditioner built from
 * the Schur complement approximation.  Level 0 is D on the lattice; each
 * level is partitioned with the all-even coarse set (Type I) and the next
 * level is its Schur complement approximation, which on that set is again a
 * Wilson operator: D_bb - D_br D_rb / d = (1/d) D_W(V, d^2 - 4) on the coarse
 * lattice, d = 4 + m, V_mu(c) = U_mu(2c) U_mu(2c + mu) (the second-order
 * formula of section 3 reduces to it on this set).  One cycle on level k:
 * y = A_rr^{-1} f_r, g = f_b - A_br y, x_b = cycle(k + 1, g),
 * x_r = A_rr^{-1}(f_r - A_rb x_b), with the A_rr solves by BiCGstab to
 * drr_tol (section 4 used one percent) and the top level solved to top_tol
 * ("inverted exactly").  With perm = GRG_PERM_I and inverse = 0 the cycle uses
 * Type I at every level (2 or 3 levels).  Any other ordering of section 2
 * (Type II, or the inverse permutations section 4's runs used, whose
 * recursion to further levels the paper does not state) gives a two-level
 * cycle: the partition of that ordering on the lattice, and on top the
 * section 3 approximation S~_bb of its Schur complement (grg_reusken_apply,
 * matrix-free) solved by BiCGstab to top_tol. */
typedef struct grg_vcycle_s *grg_vcycle;

typedef struct {
    int levels;        /* 2 or 3 (default 3): every extent must be divisible by 2^levels */
    double drr_tol;    /* relative accuracy of the A_rr solves in the cycle (default 1e-2) */
    double top_tol;    /* relative accuracy of the top level's solve (default 1e-12) */
    int max_rhs;       /* largest nrhs per call (default 12, <= 16) */
    int max_iter;      /* cap on the iterations of each BiCGstab solve (default 10000) */
    int perm;          /* ordering of the partition: GRG_PERM_I (default) or GRG_PERM_II */
    int inverse;       /* nonzero: the inverse permutation of that type (default 0); any
                          ordering but Type I needs levels = 2 */
} grg_vcycle_params;

typedef struct {
    int iters;             /* outer BiCGstab iterations */
    int converged;         /* every RHS reached tol */
    double rate;           /* average convergence rate R: the mean over RHS of
                              (|r_n| / |r_0|)^(1/n), the geometric mean of the ratio of
                              each iteration's residual to the previous one */
    double true_rel_resid; /* max over RHS of |f - D x| / |f|, recomputed */
    double t_ms;
    int cycles;            /* V-cycle applications */
} grg_vcycle_stats;

grg_status grg_vcycle_params_default(grg_vcycle_params *p);
/* Build the hierarchy on lat (gauge field set) for mass m0: the coarse
 * lattices, their blocked links and masses m_{k+1} = (4 + m_k)^2 - 4 with
 * the scale of each level (Type I), or the partition and its D_rr solver
 * (other orderings).  GRG_EINVAL if an extent is not divisible by 2^levels
 * (Type I; other orderings: by 2), if levels is not 2 for an ordering other
 * than Type I, for an unknown perm, or if 4 + m0 = 0.  lat must outlive the
 * handle. */
grg_status grg_vcycle_create(grg_lattice lat, double m0, const grg_vcycle_params *params,
                             grg_vcycle *out);
grg_status grg_vcycle_destroy(grg_vcycle v);
/* x = M f: one V-cycle on level 0 for nrhs canonical lattice fields (device). */
grg_status grg_vcycle_apply(grg_vcycle v, const double *f, double *x, int nrhs);
/* Solve D x = f (all sites, FP64) to ||f - D x|| <= tol ||f|| per RHS by
 * BiCGstab, right-preconditioned by the V-cycle when precondition != 0 (each
 * iteration applies D twice and, preconditioned, the cycle twice); x starts
 * from zero.  Canonical device fields.  stats may be NULL.  GRG_ENOCONV after
 * max_iter iterations keeps the last iterate. */
grg_status grg_vcycle_solve(grg_vcycle v, int precondition, double tol, const double *f, double *x,
                            int nrhs, grg_vcycle_stats *stats);

/* ---------------------------------------------------------------------------
 * Learned preconditioner.  M is a linear, gauge-covariant network of three
 * parallel-transport convolutions with 4 -> 8 -> 8 -> 4 colour-vector channels
 * (12 -> 24 -> 24 -> 12 complex per site; the spin index of a Dirac field is
 * the channel):  Y_f(x) = sum_h sum_f' W_h[f, f'] (T_h X_f')(x) over the hops
 * h = 0, +x, -x, +y, -y, +z, -z, +t, -t, with T_0 = 1,
 * T_{+mu} X(x) = U_mu(x) X(x + mu), T_{-mu} X(x) = U_mu(x - mu)^+ X(x - mu).
 * No bias, no activation.  Weights are complex, 9 * (32 + 64 + 32) = 1152 of
 * them, stored layer by layer as [hop][f_out][f_in] (interleaved re, im
 * doubles).  Activations and weights enter the matrix cores as bfloat16 with
 * FP32 accumulation.  Inputs are read on the rest sites only and outputs are
 * zero on the coarse sites, so M approximates D_rr^{-1}.
 * ------------------------------------------------------------------------- */
#define GRG_PRECOND_WEIGHTS 1152

/* A network bound to s (its lattice, links and coarse sites), workspaces for
 * s's max_rhs, weights zero except W_0 of every layer = identity on the
 * first channels (so M starts as the identity on Dirac fields). */
grg_status grg_precond_create(grg_schur s, grg_precond *out);
grg_status grg_precond_destroy(grg_precond p);
/* Host arrays of GRG_PRECOND_WEIGHTS complex (2 doubles each). */
grg_status grg_precond_set_weights(grg_precond p, const double *w);
grg_status grg_precond_get_weights(grg_precond p, double *w);
/* out = M in for nrhs canonical lattice fields (device). */
grg_status grg_precond_apply(grg_precond p, const double *in, double *out, int nrhs);
/* Loss L = (1/B) sum_i |M r_i - e_i|^2 / |e_i|^2 over nrhs = B pairs of
 * canonical lattice fields (device) and its Wirtinger gradient dL/dconj(W)
 * (host, GRG_PRECOND_WEIGHTS complex; the gradient of the real and imaginary
 * parts is twice its real and imaginary parts). */
grg_status grg_precond_loss_grad(grg_precond p, const double *r, const double *e, int nrhs,
                                 double *loss, double *grad);
/* Train on the GPU: each step draws `batch` random errors e_0 on the rest
 * sites, runs k minimal-residual steps of the solver on D_rr x = D_rr e_0
 * (k uniform in 0..max_mr_steps), takes the pairs (r_k, e_k = e_0 - x_k) the
 * solver produced, and applies one Adam step to the loss above. */
grg_status grg_precond_train(grg_precond p, const grg_train_params *tp, grg_train_stats *st);
/* Versioned binary weight file (magic, version, channel shape, seed, steps). */
grg_status grg_precond_save(grg_precond p, const char *path);
grg_status grg_precond_load(grg_precond p, const char *path);
/* Use p as the right preconditioner of s's inner GCR (NULL detaches).  An
 * inner solve that fails to converge or meets a non-finite value with the
 * preconditioner is redone with plain GCR, which also judges the result
 * through the FP64 residual of the defect correction. */
grg_status grg_schur_attach_precond(grg_schur s, grg_precond p);

/* ---------------------------------------------------------------------------
 * Many independent lattices at once (the batched workload of 48 lattices of
 * mixed sizes: the S_bb of section 1 for each, solved together).  The
 * members (each with its own extents, boundary signs, m0, links and
 * ordering) are concatenated in one site index and every kernel covers all
 * of them in one launch, with per-(member, RHS) step lengths.  Convergence is
 * decided on the device: per-system flags, set by the reductions and by a
 * control kernel, gate every kernel (converged systems are skipped, a launch
 * with no system left returns at once), so the whole apply -- every outer
 * defect-correction step with its inner iterations, the recomputed final
 * residual and the combine -- is one sequence of launches with no host
 * decision inside, captured once as a HIP graph on the batch's own stream
 * and replayed as one launch.  Each member's volume must be a multiple of
 * 256 sites.
 * ------------------------------------------------------------------------- */
typedef struct grg_batch_s *grg_batch;

typedef struct {
    int32_t dims[4];
    int32_t bc[4];
    double m0;
    const double *links;  /* host, canonical [V][4][3][3] complex128 */
    const int32_t *q;     /* host ordering (V entries), coarse sites first */
    int32_t n_coarse;
} grg_batch_member;

/* params->inner / inner_tol / tol / max_iter / max_outer as for one lattice;
 * check_every = inner iterations between the host's reads of the flags in
 * the eager mode; the inner solve is minimal residual (params->method other
 * than 0 gives GRG_EUNSUPPORTED; restart is not used): with params->eo and
 * every extent of every member even, on the even-odd reduced system of each
 * lattice's D_rr (d - H_pq H_qp / d on the parity with fewer rest sites, as
 * grg_reduced_apply; the same block elimination as S_bb applied to D_rr),
 * the other parity reconstructed after each inner solve; else on D_rr.
 * stream: the caller's stream, waited on at entry and made to wait for the
 * result at exit. */
grg_status grg_batch_create(const grg_batch_member *members, int count, int nrhs,
                            const grg_solver_params *params, void *stream, grg_batch *out);
grg_status grg_batch_destroy(grg_batch b);
/* Coarse vectors of the whole batch are one device array: member i's block
 * [nrhs][12 N_b(i)] complex128 starts at complex offset *offset; member ==
 * count gives the total length and total N_b. */
grg_status grg_batch_layout(grg_batch b, int member, int64_t *offset, int32_t *n_coarse);
/* y_b = S_bb x_b for every member and RHS.  use_graph = 1: one replay of the
 * captured apply (see grg_batch_graph_info; x_b and y_b pass through staging
 * buffers of the batch by two device copies), then one read of the residuals;
 * an apply the captured counts did not finish continues eagerly from there
 * and the next apply is re-captured with one more outer step.  use_graph = 0
 * launches the same kernels eagerly, the host reading the flags every
 * check_every inner iterations: same systems, same iterations, same bits. */
grg_status grg_batch_apply(grg_batch b, const double *x_b, double *y_b, int use_graph,
                           grg_solver_stats *stats);
/* Time the batched stencil launch shapes and keep the fastest (the next
 * captured apply is re-captured with them). */
grg_status grg_batch_tune(grg_batch b);
/* The shape of the captured apply: counts[0] outer defect-correction steps,
 * counts[1] inner iterations per step ({0, 0} while none is captured).  An
 * apply with use_graph = 1 runs eagerly while the batch has no recorded
 * counts (its first apply), records them, and later ones replay the graph. */
grg_status grg_batch_graph_info(grg_batch b, int32_t counts[2]);
/* The batched stencil launch in use for a precision, info = {sites per
 * workgroup, RHS per thread, workgroups}, and from the last grg_batch_tune
 * the time per launch (HIP events on the batch's stream, every system
 * active) of the stencil the solve runs in that precision (ms[0]: for the
 * inner precision with the even-odd reduced solve, one half-step of the
 * reduced operator on the compact fields, the average of its two halves)
 * and, for the inner precision, of the MR update (ms[1], on the compact
 * fields with the reduced solve); -1 where not timed. */
grg_status grg_batch_tune_info(grg_batch b, int precision, int32_t info[3], float ms[2]);

/* Kernel timing: with profiling on (on = 1), every dslash launch and every
 * phase of the solve is bracketed by HIP events on the lattice stream, and
 * the events are read at the end of each call (the phase times of
 * grg_solver_stats); with on = 2 only the stencil launches (slots 0..5) are
 * bracketed and their events are read by grg_profile_read and
 * grg_profile_reset (which first wait for the lattice stream), or at the end
 * of a call once half of the 16384 event pairs are in use, so that a timed
 * sequence of calls carries fewer events and no per-call readback; the
 * stats' phase times are then -1.  on = 0 turns profiling off; other values
 * are GRG_EINVAL.  grg_profile_read returns the count and the summed
 * milliseconds since the last reset, per slot: 0..2 full-lattice stencil
 * launches in that grg_precision, 3..5 the half-lattice stencils of the
 * even-odd reduced solve in precision - 3, 6 the FP64 defect-correction
 * steps, 7 the Krylov vector kernels, 8 the learned preconditioner's
 * applications. */
grg_status grg_profile_enable(grg_schur s, int on);
grg_status grg_profile_read(grg_schur s, int precision, int64_t *count, double *total_ms);
grg_status grg_profile_reset(grg_schur s);

#ifdef __cplusplus
}
#endif
#endif /* GRG_H */
