/*
 * marnoldi.h -- C interface of the MI355X (gfx950) multiple Arnoldi library.
 *
 * The library computes, for every requested column j of a sparse
 * real-symmetric tight-binding pencil (H, S) with S positive definite, the
 * column j of the density matrix rho and of the energy-density matrix pi of
 * the multiple Arnoldi method (Hoshi, Yamamoto, Fujiwara, Sogabe, Zhang,
 * arXiv:1202.0098, Sec. 2):
 *
 *   s_j = S^-1 e_j by an inner conjugate-gradient loop          (Sec. 2)
 *   L_j = K_p(H; e_j) + K_q(H; s_j), an S-orthonormal basis     (Eqs. 4-9)
 *   (H~, S~) = (U^T H U, U^T S U), eigenpairs (eps_a, C_a)      (Galerkin, Eq. 10)
 *   rho_ij = sum_a f(eps_a) v_ia v_ja, pi_ij = sum_a f eps_a v_ia v_ja  (Eqs. 13-14)
 *   E_j = sum_i rho_ij H_ji, N_j = sum_i rho_ij S_ji           (Eq. 17; Tr rho S)
 *
 * with H and S restricted to a real-space region around the atom of j
 * (the real-space projection of Sec. 3) and f the Fermi-Dirac function at
 * temperature kT and chemical potential mu; mu is found by bisection on the
 * electron count when not given (Sec. 2, summation over j).
 *
 * Conventions
 *   - Matrices are atom-block CSR with a uniform number o of orbitals per
 *     atom: block k of block-row A couples atom A (rows) and atom blk_col[k]
 *     (columns); its o*o values are row-major.  The block pattern must be
 *     structurally symmetric, contain every diagonal block, and H, S must be
 *     symmetric (block (B,A) equals the transpose of block (A,B)).
 *   - A column j is a global orbital index; atom(j) = j / o, orbital j % o.
 *   - Outputs rho and pi use the same block-slot layout as the input: slot
 *     (k, r, c) of block k in block-row A holds element (i, j) with
 *     j = (A, r), i = (blk_col[k], c).  Block-row A therefore stores the
 *     columns j of atom A, restricted to the pattern of H (only these elements
 *     are needed, Sec. 2 after Eq. 18).
 *   - rho, pi, E_j and N_j are per spin; ma_result.energy and n_elec are
 *     multiplied by opts.spin.
 *   - All functions return an ma_status; no exception crosses the interface.
 *     On error, ma_last_error() describes it.
 *   - Device work is enqueued on the stream given to ma_create.  If that is
 *     the null stream (which cannot be captured into a hipGraph), the solve
 *     runs on a stream of the library's own, ordered after the work already
 *     queued on the null stream.  Every function returns after its device
 *     work has completed.
 *   - One context per host thread; contexts are independent.
 */
#ifndef MARNOLDI_H
#define MARNOLDI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MA_API __attribute__((visibility("default")))

#define MA_MAX_ORB 16   /* largest o supported */
#define MA_MAX_NU 64    /* largest p + q supported */

typedef struct ma_ctx ma_ctx;

typedef enum {
    MA_OK = 0,
    MA_EINVAL = -1,   /* invalid argument or input (nothing was launched) */
    MA_ENOMEM = -2,   /* device or host allocation failed */
    MA_EDEVICE = -3,  /* a HIP call failed */
    MA_ENOTPD = -4,   /* CG met non-positive curvature: S_A not positive definite */
    MA_ENOCONV = -5,  /* CG did not reach opts.cg_tol */
    MA_ESTATE = -6    /* call out of order (e.g. solve before build_system) */
} ma_status;

enum { MA_REGION_ALL = 0, MA_REGION_RADIUS = 1, MA_REGION_NEAREST = 2 };
enum { MA_PREC_FP64 = 0, MA_PREC_MIXED = 1, MA_PREC_MIXED_F64ACC = 2 };
enum { MA_START_ZERO = 0, MA_START_LEARNED = 1, MA_START_PREVIOUS = 2 };
enum { MA_BASIS_AUTO = 0, MA_BASIS_ONCHIP = 1, MA_BASIS_WORKSPACE = 2, MA_BASIS_GROUP = 3,
       MA_BASIS_ATOM = 4 };

/* The pencil and its geometry.  All pointers are host memory owned by the
 * caller; ma_build_system copies what it needs. */
typedef struct {
    int32_t n_atoms;
    int32_t n_orb;             /* o, orbitals per atom, 1..MA_MAX_ORB */
    const int64_t *blk_ptr;    /* n_atoms + 1 block-row offsets */
    const int32_t *blk_col;    /* nblk column atoms, ascending in each row */
    const double *H;           /* nblk * o * o */
    const double *S;           /* nblk * o * o */
    const double *xyz;         /* n_atoms * 3 positions (Angstrom); may be NULL for MA_REGION_ALL */
    const double *box;         /* 3 orthorhombic periodic box lengths; NULL = open boundaries */
} ma_system;

/* Real-space region of each atom (Sec. 3, projection of H and S).
 * ALL: the whole system.  RADIUS: atoms with minimum-image squared distance
 * below radius^2.  NEAREST: the n_rp (or n_rp_atom[A]) nearest atoms, atom A
 * included, ties broken by the lower atom index.  Every region must contain
 * the pattern of its atom's block-row (else MA_EINVAL). */
typedef struct {
    int32_t mode;
    double radius;
    int32_t n_rp;
    const int32_t *n_rp_atom;  /* optional, n_atoms entries (host) */
} ma_region;

typedef struct {
    int32_t precision;      /* MA_PREC_FP64: everything FP64.  MA_PREC_MIXED:
                               FP32 SpMV and CG with FP32 accumulation, FP64
                               residual judge and refinement, FP64 Gram-Schmidt,
                               projection and eigensolve.  MA_PREC_MIXED_F64ACC:
                               as MIXED, but the basis SpMVs read FP32 operator
                               values into FP64 vectors and accumulators. */
    double cg_tol;          /* stop when ||e_j - S_A s_j||_2 <= cg_tol (default 1e-12) */
    double inner_tol;       /* mixed: relative residual of each FP32 CG pass (default 1e-6;
                               a pass whose start residual is small stops once the
                               residual is cg_tol / 10) */
    int32_t max_refine;     /* mixed: FP64 refinement rounds (default 8) */
    double breakdown_tau;   /* a basis candidate is dropped when its S-norm after
                               orthogonalisation is <= tau * its S-norm before (1e-10) */
    double spin;            /* spin degeneracy for energy and n_elec (default 2) */
    double n_target;        /* per-spin electron count sum_j N_j for the bisection
                               (used when mu is NaN; default: half of M) */
    int32_t start;          /* MA_START_ZERO; MA_START_LEARNED (needs a model);
                               MA_START_PREVIOUS: the s_j of the same column kept by an
                               earlier solve with keep_sj (possibly of an earlier
                               geometry of the same atoms, after ma_build_system),
                               mapped onto the current region atom by atom (atoms that
                               left the region are dropped, new ones start at zero);
                               like the learned start, judged by the FP64 residual */
    int32_t slots_per_cu;   /* persistent workgroups per compute unit (0 = the
                               autotuned value for this (p, q, precision) if
                               ma_autotune ran, else the occupancy limit) */
    int32_t schedule;       /* column-to-workgroup schedule, MA_SCHED_*; -1 = autotuned
                               value if available, else MA_SCHED_LPT */
    int32_t use_graph;      /* 1: capture the launch sequence in a hipGraph and replay it
                               while the configuration and buffers are unchanged */
    int32_t basis_kernel;   /* MA_BASIS_AUTO: the autotuned kernel for (p, q, precision)
                               if ma_autotune ran, else MA_BASIS_WORKSPACE.
                               MA_BASIS_WORKSPACE: one column per workgroup, basis in a
                               device workspace, one dot sweep and one update sweep per
                               basis vector.
                               MA_BASIS_ONCHIP: one column per workgroup, basis in LDS
                               and registers (regions of at most 512 orbitals,
                               p + q <= 32, q <= 16; q <= 8 when p + q <= 16).
                               MA_BASIS_GROUP: the requested columns of one atom in
                               lockstep, one SpMM per step for all of them (o = 4 or
                               9).
                               MA_BASIS_ATOM: the requested columns of one atom in
                               lockstep, every operator pass one block SpMM over a
                               staged set of their vectors, bases in a device
                               workspace (o = 4 or 9; MA_PREC_FP64 and
                               MA_PREC_MIXED_F64ACC).  A forced kernel that cannot
                               hold the shape is MA_EINVAL. */
    int32_t chunk_columns;  /* columns per chunk of the processing order (0 = as many
                               as a 4 GiB chunk buffer holds); a solve of several
                               chunks launches eagerly instead of replaying graphs */
    int32_t pipeline;       /* >= 2: a solve of at least 2048 * pipeline columns is cut
                               into pipeline + 2 chunks of geometrically falling size
                               (equal chunks where the 4 GiB chunk buffer caps the
                               first), and the eigensolver of chunk k runs on a second
                               stream beside the later basis kernels, with a ring of
                               chunk buffers of at most 8 GiB; 0 or 1: off (chunks in
                               sequence on one stream); -1 (default): the autotuned
                               choice for (p, q, precision) if ma_autotune ran, else 4 */
    int32_t keep_sj;        /* 1: keep each solved column's s_j = S_A^-1 e_j (region
                               vector, FP64, M * nmax doubles in all) for a later solve
                               with MA_START_PREVIOUS; the kept set belongs to the
                               geometry of the solve that wrote it (default 0) */
} ma_opts;

/* Schedules of the persistent column kernel.  LPT: one queue, columns with
 * the largest region first.  INPUT: one queue in the caller's order.
 * XCD_INPUT / XCD_LPT: the (caller-ordered or LPT-ordered) list cut into one
 * contiguous chunk per XCD; workgroup b serves chunk b % 8 first (workgroups
 * are dispatched to the 8 XCDs round-robin), then steals from the others, so
 * spatially adjacent columns share an XCD's L2.  SPATIAL: one queue, the atoms
 * of each chunk in Morton order of their positions (cells of two mean atomic
 * spacings; index order without positions), so that the columns in flight
 * together have overlapping regions and share their operator blocks in the
 * caches (real-space projection, Sec. 3). */
enum { MA_SCHED_LPT = 0, MA_SCHED_INPUT = 1, MA_SCHED_XCD_INPUT = 2, MA_SCHED_XCD_LPT = 3,
       MA_SCHED_SPATIAL = 4 };

/* Outputs of ma_solve_columns.  Device pointers are optional (NULL = not
 * written) and owned by the caller. */
typedef struct {
    double *rho;            /* device, nblk*o*o, block-slot layout; only the rows
                               of the solved columns are written */
    double *pi;             /* device, same layout */
    double *eps;            /* device, ncols*(p+q): Ritz values ascending, NaN padded */
    double *wts;            /* device, ncols*(p+q): w_a = v_ja (S v_a)_j */
    int32_t *col_stats;     /* device, ncols*8: nu_eff, CG iterations, FP64
                               residual evaluations, status, start used (0 zero,
                               1 learned, 2 learned but rejected by the residual
                               judge, 3 previous, 4 previous but rejected), 3
                               reserved */
    double energy;          /* spin * sum_j E_j over the solved columns */
    double n_elec;          /* spin * sum_j N_j over the solved columns */
    double mu;              /* chemical potential used */
    double elapsed_ms;      /* device time of the whole solve on the stream */
    double kernel_ms;       /* device time of the basis kernel alone (CG, basis,
                               Galerkin pair; HIP events around its launches on the
                               same stream, summed over column chunks) */
    float *sj_near;         /* device, ncols*12*o, optional: the converged s_j on the
                               orbitals of the 12 atoms nearest to atom(j), nearest
                               first (atom(j) itself first), the start network's
                               training target */
    double eig_ms;          /* device time of the batched reduced-eigenproblem kernel */
} ma_result;

/* Result of ma_autotune. */
typedef struct {
    int32_t slots_per_cu;       /* chosen */
    int32_t schedule;           /* chosen */
    double best_ms;             /* whole-solve device time of the chosen configuration */
    int32_t n_tried;
    int32_t tried_slots[64];
    int32_t tried_schedule[64];
    double tried_ms[64];        /* whole-solve device time of each candidate (best of reps) */
    int32_t basis_kernel;       /* chosen: MA_BASIS_ONCHIP, _WORKSPACE, _GROUP or _ATOM */
    int32_t tried_kernel[64];
    int32_t pipeline;           /* chosen: the pipeline option of the solve (0 = off) */
    int32_t tried_pipeline[64];
} ma_tuning;

/* Library version string (static storage). */
MA_API const char *ma_version(void);

/* Fill *o with the defaults listed above (NULL: no-op). */
MA_API void ma_default_opts(ma_opts *o);

/* Create a context on HIP device `device` that enqueues on `stream` (a
 * hipStream_t, e.g. torch.cuda.current_stream().cuda_stream; NULL = the null
 * stream).  The context owns every device buffer it allocates; *out is NULL
 * on failure (MA_EDEVICE: no such device or a HIP call failed). */
MA_API ma_status ma_create(ma_ctx **out, int32_t device, void *stream);

/* Free every resource of the context (MA_EINVAL for NULL). */
MA_API ma_status ma_destroy(ma_ctx *ctx);

/* Description of the last error on this context (never NULL; owned by the
 * context, valid until its next call). */
MA_API const char *ma_last_error(const ma_ctx *ctx);

/* Load the pencil (H, S) of Sec. 2 -- H real symmetric, S symmetric positive
 * definite, both sparse in the atom-block pattern -- and build the real-space
 * region of every atom (Sec. 3, the projection of H and S onto a sphere or
 * the N_RP nearest atoms around the atom of basis j) with its local block
 * operators H_A, S_A (principal submatrices, addressed through a local block
 * index: the values are not copied per region).  Host arrays are copied;
 * FP64 and FP32 copies of H and S are uploaded.  Replaces any previous system
 * of the context.  MA_EINVAL (nothing uploaded) on a malformed pattern,
 * asymmetric or non-finite values, unsupported o, or a region that misses
 * part of its atom's pattern. */
MA_API ma_status ma_build_system(ma_ctx *ctx, const ma_system *sys, const ma_region *reg);

/* Sizes of the built system (Sec. 3 regions): M, nblk, the largest region
 * dimension and the largest number of pattern rows of a column; any output
 * pointer may be NULL.  MA_ESTATE before a successful build. */
MA_API ma_status ma_system_info(const ma_ctx *ctx, int64_t *M, int64_t *nblk,
                                int32_t *max_region_orbitals, int32_t *max_pattern_rows);

/* Per-atom sizes of the real-space regions (Sec. 3) of the built system
 * (host arrays of n_atoms entries, either may be NULL): the number of atoms
 * in the atom's region and the number of blocks of its local operator H_A
 * (the same pattern serves S_A). */
MA_API ma_status ma_region_sizes(const ma_ctx *ctx, int32_t *region_atoms,
                                 int64_t *local_blocks);

/* Host-only query (no device is used): the region of `atom` (Sec. 3,
 * real-space projection) that ma_build_system would build for (sys, reg),
 * ascending atom indices, written to out[0..min(count, cap)) (host, caller
 * owned).  Returns the region's atom count, or a negative ma_status on
 * invalid arguments. */
MA_API int64_t ma_region_atoms(const ma_system *sys, const ma_region *reg, int32_t atom,
                               int32_t *out, int64_t cap);

/* The per-column multiple Arnoldi solve (Sec. 2): for every column j of
 * cols[0..ncols) (host array of global orbital indices; NULL = all M columns,
 * in order) the inner CG for s_j = S_A^-1 e_j, the S-orthonormal basis of
 * K_p(H; e_j) + K_q(H; s_j) (Eq. 4, built by Eqs. 6-9), the Galerkin pair and
 * its eigenpairs (Eq. 10), and rho_ij, pi_ij (Eqs. 13-14) with E_j, N_j
 * (Eq. 17 and Tr rho S), at temperature kT > 0 and chemical potential mu
 * (NaN: bisect so that sum_j N_j = opts->n_target over the solved columns,
 * Sec. 2, electron count summed over j).  p >= 1, q >= 0, p + q <=
 * MA_MAX_NU; opts NULL = defaults.  Outputs go to the caller's device
 * pointers in *out (any may be NULL) and the scalars of *out.  Breakdowns are
 * not errors (see col_stats).  Returns MA_ENOTPD / MA_ENOCONV if some
 * column's CG failed (the first such column is named by ma_last_error);
 * outputs are then undefined for that column.  A bisected solve keeps its
 * Ritz data and amplitudes for ma_find_mu until the next solve. */
MA_API ma_status ma_solve_columns(ma_ctx *ctx, int64_t ncols, const int32_t *cols,
                                  int32_t p, int32_t q, double mu, double kT,
                                  const ma_opts *opts, ma_result *out);

/* Chemical potential again (Sec. 2: mu fixed by the electron count summed
 * over the basis index j), on the Ritz values, weights and amplitudes of the
 * last solve, which must have bisected mu (else MA_ESTATE): K-section on
 * sum_j sum_a f((eps_a - mu)/kT) w_a = n_target (per spin), then rho and pi
 * (Eqs. 13-14, into out->rho / out->pi, device, same layout as the solve,
 * either may be NULL; only the solved columns' rows are written) and
 * out->energy, out->n_elec (times `spin`), out->mu, out->elapsed_ms.  kT may
 * differ from the solve's: the amplitudes do not depend on it.  No column is
 * re-solved.  If the solve wrote its Ritz data to the caller's eps/wts
 * buffers (or into a caller workspace), those must still hold them. */
MA_API ma_status ma_find_mu(ma_ctx *ctx, double n_target, double kT, double spin,
                            ma_result *out);

/* Atomic forces from the column outputs (Sec. 2: F_K as the sum over j of
 * the partial sums F_K^(j), which involve rho_ij and pi_ij only at pattern
 * elements):
 *   F_K = -spin sum_j sum_i [rho_ij dH_ji/dR_K - pi_ij dS_ji/dR_K].
 * dH, dS: device, nblk * 3 * o * o FP64 (block k, Cartesian direction d,
 * then the o x o block row-major): the derivative of block k = (A, B) of H
 * (resp. S) with respect to the position of its column atom B; its
 * derivative with respect to R_A is taken as the negative (translation
 * invariance), and the atom-diagonal blocks are not used.  rho, pi: device,
 * nblk * o * o, the outputs of ma_solve_columns (every column whose pattern
 * reaches an atom must have been solved for that atom's force).  forces:
 * device, n_atoms * 3, written.  The overlap term enters with the sign of
 * the derivative of the grand potential for S-normalised eigenvectors.
 * All arrays are caller owned; MA_ESTATE before a build. */
MA_API ma_status ma_forces(ma_ctx *ctx, const double *dH, const double *dS, const double *rho,
                           const double *pi, double spin, double *forces);

/* Density of states of the last solve's subspaces (the subspace Green's
 * functions of Eqs. 11-12 traced with the overlap, Lorentzian broadening eta
 * > 0): dos[k] = spin/pi sum_j sum_a w_a eta / ((E_k - eps_a)^2 + eta^2)
 * with w_a = v_ja (S v_a)_j, over the columns of the last solve.  energies
 * and dos: host, n_energies entries (caller owned).  MA_ESTATE if no solve
 * has run since the last build (or the last one failed or was allocation-free). */
MA_API ma_status ma_dos(ma_ctx *ctx, int64_t n_energies, const double *energies, double eta,
                        double spin, double *dos);

/* The subspace Green's function at complex energy z (Eq. 12) applied to e_j
 * (Eq. 11), G_ij(z) = sum_a v_ia v_ja / (z - eps_a), at the pattern
 * elements of every column of the last solve, which must have bisected mu
 * (its amplitudes are reused; else MA_ESTATE).  g_re, g_im: device, nblk *
 * o * o, the block-slot layout of rho (either may be NULL; only the solved
 * columns' rows are written).  Im z must be nonzero. */
MA_API ma_status ma_green(ma_ctx *ctx, double z_re, double z_im, double *g_re, double *g_im);

/* Bytes of device workspace a solve with these arguments (the arguments of
 * ma_solve_columns; only whether mu is NaN matters) needs when the caller
 * provides it: the column lists, the basis workspace of the persistent
 * workgroups, the chunk buffers, Ritz data, amplitudes (bisected solves),
 * statistics and the reduction scratch.  0 on invalid arguments
 * (ma_last_error says why).  An upper bound: buffers the caller passes in
 * ma_result (eps, wts, col_stats) are counted as if the library held them. */
MA_API size_t ma_workspace_size(ma_ctx *ctx, int64_t ncols, const int32_t *cols, int32_t p,
                                int32_t q, double mu, const ma_opts *opts);

/* Use [device_ptr, device_ptr + bytes) (caller owned, 256-byte aligned,
 * device memory of the context's device) for the per-solve buffers of the
 * following solves and autotuning instead of the library's own allocations;
 * NULL, 0 goes back to them.  A solve that needs more than `bytes` fails with
 * MA_EINVAL naming the size it needs.  The workspace must stay valid while a
 * solve runs and, for ma_find_mu, until the next solve.  The system (H, S,
 * regions) stays in the library's own memory. */
MA_API ma_status ma_set_workspace(ma_ctx *ctx, void *device_ptr, size_t bytes);

/* ------------------------------------------------------------------------
 * Learned CG start (callers that want fewer CG iterations).  A 3-layer
 * perceptron (width 256, SiLU) maps a column's descriptor -- for each of the
 * 48 atoms nearest to atom(j), excluding it, nearest first: |d|/5 A and the
 * unit vector d/|d| -- plus the one-hot orbital of j (n_in = 192 + o) to the
 * coefficients of s_j on the orbitals of the 12 atoms nearest to atom(j)
 * (n_out = 12 o).  Inference runs in BF16 on the matrix cores with FP32
 * accumulation; training runs in FP32.  In a solve with MA_START_LEARNED the
 * prediction is the CG start unless the FP64 residual ||S_A x0 - e_j|| is
 * not below ||e_j|| = 1, in which case the column starts from zero.
 * Descriptors need positions in ma_system.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_in, n_hidden, n_out;
    int64_t n_params;   /* W1 (n_in x n_hidden), b1, W2 (n_hidden^2), b2, W3 (n_hidden x n_out), b3 */
} ma_mlp_shape;

/* Shape of the start network for the built system (MA_ESTATE before a
 * build).  The network is not part of the paper's method: it only supplies
 * the start vector of the inner CG of Sec. 2, whose result it does not
 * change beyond the CG tolerance. */
MA_API ma_status ma_mlp_shape_of(const ma_ctx *ctx, ma_mlp_shape *out);

/* Random initial weights (He-scaled normal, zero biases, seeded) and zeroed
 * Adam state; the network becomes the context's start model (the CG start
 * of Sec. 2).  MA_ESTATE before a build. */
MA_API ma_status ma_mlp_init(ma_ctx *ctx, uint64_t seed);

/* Copy the start network's parameters (host, FP32, caller owned, the packed
 * order of ma_mlp_shape) in/out; MA_EINVAL if count != n_params. */
MA_API ma_status ma_mlp_set_params(ma_ctx *ctx, const float *params, int64_t count);
MA_API ma_status ma_mlp_get_params(const ma_ctx *ctx, float *params, int64_t count);

/* Descriptors of cols[0..ncols) (host list) into feat (device, caller owned,
 * ncols * n_in FP32): the local geometry around atom(j) that the start
 * network reads (needs positions in ma_system). */
MA_API ma_status ma_column_features(ma_ctx *ctx, int64_t ncols, const int32_t *cols, float *feat);

/* y = net(x) for n rows (device arrays, caller owned, n * n_in -> n * n_out,
 * FP32); bf16 = 1 uses the inference kernel (BF16 matrix cores, FP32
 * accumulation), 0 the FP32 training path. */
MA_API ma_status ma_mlp_forward(ma_ctx *ctx, const float *x, int64_t n, float *y, int32_t bf16);

/* Mean squared error of the start network over n rows (rows idx[i] of x and
 * t, device tables of n_rows rows, if idx != NULL, else rows 0..n-1) and its
 * gradient (host, n_params floats, may be NULL).  The gather checks the device
 * indices: one outside [0, n_rows) fails the call with MA_EINVAL. */
MA_API ma_status ma_mlp_loss_grad(ma_ctx *ctx, const float *x, const float *t, int64_t n_rows,
                                  const int32_t *idx, int64_t n, double *loss, float *grad);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8) of the start network on the
 * mean squared error of the n rows idx[i] (device int32, NULL = rows
 * 0..n-1) of x and t (device tables of n_rows rows); the loss before the step
 * in *loss.  An index outside [0, n_rows) fails the call with MA_EINVAL
 * before the parameters change. */
MA_API ma_status ma_mlp_train_step(ma_ctx *ctx, const float *x, const float *t, int64_t n_rows,
                                   const int32_t *idx, int64_t n, float lr, double *loss);

/* Autotuner of the launch (not part of the paper's method, which runs the
 * columns of Sec. 2 independently): time the solve on cols[0..ncols) (NULL = all) for every
 * candidate -- basis kernel (each one that can hold the shape) x
 * slots per CU from 1 to that kernel's occupancy limit x every schedule, with
 * the pipeline option of opts (-1: 4), and each kernel's fastest slots per
 * CU again with pipelining off, every schedule --
 * `reps` times each at chemical potential mu (finite), and keep the fastest
 * configuration for this (p, q, opts->precision) in the context, except that
 * when cols is a proper subset of the columns, among trials of its kernel,
 * slots and pipelining within 2 % of it the schedule is taken in the order
 * SPATIAL, INPUT, XCD_INPUT, XCD_LPT, LPT (a sample of the columns cannot
 * resolve the schedules' cache effects); solves with
 * basis_kernel = MA_BASIS_AUTO, slots_per_cu = 0, schedule = -1 and
 * pipeline = -1 then use it.  Outputs (rho, pi) are not written. */
MA_API ma_status ma_autotune(ma_ctx *ctx, int64_t ncols, const int32_t *cols, int32_t p,
                             int32_t q, double mu, double kT, const ma_opts *opts, int32_t reps,
                             ma_tuning *out);

/* Store a previously found launch tuning for (p, q, precision) (e.g. from a cache);
 * basis_kernel is MA_BASIS_ONCHIP, MA_BASIS_WORKSPACE, MA_BASIS_GROUP or MA_BASIS_ATOM
 * (MA_BASIS_AUTO keeps the automatic choice); pipeline as in ma_opts (-1: 4). */
MA_API ma_status ma_set_tuning(ma_ctx *ctx, int32_t p, int32_t q, int32_t precision,
                               int32_t slots_per_cu, int32_t schedule, int32_t basis_kernel,
                               int32_t pipeline);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve
 * of ma_solve_columns with every per-solve buffer (column lists, queues, the
 * basis workspace of the persistent workgroups, the chunk buffer, Ritz data
 * and amplitudes when not passed in *out, reduction scratch) carved from a
 * static device scratch of 256 MiB that the library holds on each device it
 * runs on until the process ends.  It calls no hipMalloc, hipFree or other
 * allocating routine; the context's system (ma_build_system) must be built.
 * The chunk buffer takes at most a quarter of the scratch (more chunks, one
 * stream, no hipGraph) and the persistent workgroups are as many as the rest
 * holds; a solve that does not fit (too many columns, too large a region or
 * subspace) fails with MA_EINVAL before any launch.  Zero CG start only;
 * sj_near must be NULL; kernel_ms and eig_ms are reported as 0.  Every call
 * on a device shares that device's scratch, which keeps the last call's
 * contents: calls that overlap on one device (several contexts or threads)
 * race.  The Ritz data of a bisected call are not kept for ma_find_mu.
 * Results equal those of ma_solve_columns to rounding.
 * ------------------------------------------------------------------------ */
MA_API ma_status ma_solve_columns_noalloc(ma_ctx *ctx, int64_t ncols, const int32_t *cols,
                                          int32_t p, int32_t q, double mu, double kT,
                                          const ma_opts *opts, ma_result *out);

#ifdef __cplusplus
}
#endif

#endif /* MARNOLDI_H */
