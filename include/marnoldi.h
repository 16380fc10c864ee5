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
enum { MA_START_ZERO = 0, MA_START_LEARNED = 1 };
enum { MA_BASIS_AUTO = 0, MA_BASIS_ONCHIP = 1, MA_BASIS_WORKSPACE = 2, MA_BASIS_GROUP = 3 };

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
    double inner_tol;       /* mixed: relative residual of each FP32 CG pass (default 1e-6) */
    int32_t max_refine;     /* mixed: FP64 refinement rounds (default 8) */
    double breakdown_tau;   /* a basis candidate is dropped when its S-norm after
                               orthogonalisation is <= tau * its S-norm before (1e-10) */
    double spin;            /* spin degeneracy for energy and n_elec (default 2) */
    double n_target;        /* per-spin electron count sum_j N_j for the bisection
                               (used when mu is NaN; default: half of M) */
    int32_t start;          /* MA_START_ZERO, or MA_START_LEARNED (needs a model) */
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
                               9).  A forced kernel that cannot hold the shape is
                               MA_EINVAL. */
    int32_t chunk_columns;  /* columns per chunk of the processing order (0 = as many
                               as a 4 GiB chunk buffer holds); a solve of several
                               chunks launches eagerly instead of replaying graphs */
    int32_t pipeline;       /* >= 2 (default 4): a solve of at least 2048 * pipeline
                               columns is cut into pipeline + 2 chunks of geometrically
                               falling size (equal chunks where the 4 GiB chunk buffer
                               caps the first), and the eigensolver of chunk k runs on
                               a second stream beside the later basis kernels, with a
                               ring of chunk buffers of at most 8 GiB (0 or 1: off) */
} ma_opts;

/* Schedules of the persistent column kernel.  LPT: one queue, columns with
 * the largest region first.  INPUT: one queue in the caller's order.
 * XCD_INPUT / XCD_LPT: the (caller-ordered or LPT-ordered) list cut into one
 * contiguous chunk per XCD; workgroup b serves chunk b % 8 first (workgroups
 * are dispatched to the 8 XCDs round-robin), then steals from the others, so
 * spatially adjacent columns share an XCD's L2. */
enum { MA_SCHED_LPT = 0, MA_SCHED_INPUT = 1, MA_SCHED_XCD_INPUT = 2, MA_SCHED_XCD_LPT = 3 };

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
                               judge), 3 reserved */
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
    int32_t basis_kernel;       /* chosen: MA_BASIS_ONCHIP, MA_BASIS_WORKSPACE or MA_BASIS_GROUP */
    int32_t tried_kernel[64];
} ma_tuning;

/* Library version string. */
MA_API const char *ma_version(void);

/* Fill *o with the defaults listed above. */
MA_API void ma_default_opts(ma_opts *o);

/* Create a context on HIP device `device` that enqueues on `stream` (a
 * hipStream_t, e.g. torch.cuda.current_stream().cuda_stream; NULL = the null
 * stream).  The context owns every device buffer it allocates. */
MA_API ma_status ma_create(ma_ctx **out, int32_t device, void *stream);

/* Free every resource of the context. */
MA_API ma_status ma_destroy(ma_ctx *ctx);

/* Description of the last error on this context (never NULL). */
MA_API const char *ma_last_error(const ma_ctx *ctx);

/* Validate the pencil, build the per-atom regions and their local block
 * operators, and upload everything (FP64 and FP32 copies) to the device.
 * Replaces any previous system of the context.  MA_EINVAL on a malformed
 * pattern, asymmetric or non-finite values, unsupported o, or a region that
 * misses part of its atom's pattern. */
MA_API ma_status ma_build_system(ma_ctx *ctx, const ma_system *sys, const ma_region *reg);

/* Sizes of the built system: M, nblk, the largest region dimension and the
 * largest number of pattern rows of a column. */
MA_API ma_status ma_system_info(const ma_ctx *ctx, int64_t *M, int64_t *nblk,
                                int32_t *max_region_orbitals, int32_t *max_pattern_rows);

/* Per-atom sizes of the built system (host arrays of n_atoms entries, either
 * may be NULL): the number of atoms in the atom's region and the number of
 * blocks of its local operator H_A (the same pattern serves S_A). */
MA_API ma_status ma_region_sizes(const ma_ctx *ctx, int32_t *region_atoms,
                                 int64_t *local_blocks);

/* Host-only query (no device is used): the region of `atom` that
 * ma_build_system would build for (sys, reg), ascending atom indices, written
 * to out[0..min(count, cap)).  Returns the region's atom count, or a negative
 * ma_status on invalid arguments.  Meant for inspecting and testing the
 * real-space projection. */
MA_API int64_t ma_region_atoms(const ma_system *sys, const ma_region *reg, int32_t atom,
                               int32_t *out, int64_t cap);

/* Solve columns cols[0..ncols) (host array of global orbital indices; NULL =
 * all M columns, in order) with subspace dimensions p >= 1, q >= 0,
 * p + q <= MA_MAX_NU, temperature kT > 0 and chemical potential mu (NaN:
 * bisect so that sum_j N_j = opts->n_target over the solved columns).
 * opts NULL = defaults.  Breakdowns are not errors (see col_stats).  Returns
 * MA_ENOTPD / MA_ENOCONV if some column's CG failed (the first such column is
 * named by ma_last_error); outputs are then undefined for that column. */
MA_API ma_status ma_solve_columns(ma_ctx *ctx, int64_t ncols, const int32_t *cols,
                                  int32_t p, int32_t q, double mu, double kT,
                                  const ma_opts *opts, ma_result *out);

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

/* Shape of the start network for the built system. */
MA_API ma_status ma_mlp_shape_of(const ma_ctx *ctx, ma_mlp_shape *out);

/* Random initial weights (He-scaled normal, zero biases, seeded) and zeroed
 * Adam state; the network becomes the context's start model. */
MA_API ma_status ma_mlp_init(ma_ctx *ctx, uint64_t seed);

/* Copy the parameters (host, FP32, the packed order of ma_mlp_shape) in/out. */
MA_API ma_status ma_mlp_set_params(ma_ctx *ctx, const float *params, int64_t count);
MA_API ma_status ma_mlp_get_params(const ma_ctx *ctx, float *params, int64_t count);

/* Descriptors of cols[0..ncols) (host list) into feat (device, ncols * n_in). */
MA_API ma_status ma_column_features(ma_ctx *ctx, int64_t ncols, const int32_t *cols, float *feat);

/* y = net(x) for n rows (device arrays, n * n_in -> n * n_out); bf16 = 1 uses
 * the inference kernel, 0 the FP32 training path. */
MA_API ma_status ma_mlp_forward(ma_ctx *ctx, const float *x, int64_t n, float *y, int32_t bf16);

/* Mean squared error over n rows (rows idx[i] of x and t if idx != NULL) and
 * its gradient (host, n_params floats, may be NULL). */
MA_API ma_status ma_mlp_loss_grad(ma_ctx *ctx, const float *x, const float *t, const int32_t *idx,
                                  int64_t n, double *loss, float *grad);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on the mean squared error of the
 * n rows idx[i] (device int32, NULL = rows 0..n-1) of x and t (device). */
MA_API ma_status ma_mlp_train_step(ma_ctx *ctx, const float *x, const float *t, const int32_t *idx,
                                   int64_t n, float lr, double *loss);

/* Autotuner: time the basis kernel on cols[0..ncols) (NULL = all) for every
 * candidate -- basis kernel (each one that can hold the shape) x
 * slots per CU from 1 to that kernel's occupancy limit x every schedule --
 * `reps` times each at chemical potential mu (finite), and keep the fastest
 * configuration for this (p, q, opts->precision) in the context; solves with
 * basis_kernel = MA_BASIS_AUTO, slots_per_cu = 0 and schedule = -1 then use
 * it.  Outputs (rho, pi) are not written. */
MA_API ma_status ma_autotune(ma_ctx *ctx, int64_t ncols, const int32_t *cols, int32_t p,
                             int32_t q, double mu, double kT, const ma_opts *opts, int32_t reps,
                             ma_tuning *out);

/* Store a previously found tuning for (p, q, precision) (e.g. from a cache);
 * basis_kernel is MA_BASIS_ONCHIP, MA_BASIS_WORKSPACE or MA_BASIS_GROUP
 * (MA_BASIS_AUTO keeps the automatic choice). */
MA_API ma_status ma_set_tuning(ma_ctx *ctx, int32_t p, int32_t q, int32_t precision,
                               int32_t slots_per_cu, int32_t schedule, int32_t basis_kernel);

#ifdef __cplusplus
}
#endif

#endif /* MARNOLDI_H */
