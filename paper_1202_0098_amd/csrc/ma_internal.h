// Internal declarations shared by the host side (ma_host.cpp) and the
// kernels (ma_kernels.hip) of libmarnoldi.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ma {

constexpr int kThreads = 256;            // workgroup size of the column kernel
constexpr int kWaves = kThreads / 64;
constexpr int kMaxNu = 64;
constexpr int kBisectTrials = 15;        // trial potentials per bisection pass
constexpr int kBisectPasses = 14;        // 16^14 = 7.2e16: any bracket narrows below 1e-15
constexpr int kCountBlocks = 1024;       // fixed grid of the electron-count kernel
constexpr int kNbDesc = 48;              // neighbours in a column descriptor
constexpr int kNbOut = 12;               // atoms whose s_j coefficients the network predicts
constexpr int kGeoFeat = 4 * kNbDesc;    // (d/5, dx/d, dy/d, dz/d) per neighbour
constexpr int kHidden = 256;             // hidden width of the start network

// Device view of a built system.
struct DevSystem {
    int o;                     // orbitals per atom
    int n_atoms;
    int nmax;                  // largest region dimension (orbitals)
    int maxpat;                // largest pattern rows of a column (blocks * o)
    const int64_t *blk_ptr;    // n_atoms + 1
    const int32_t *blk_col;    // nblk
    const double *Hd, *Sd;     // FP64 values, nblk * o * o
    const float *Hf, *Sf;      // FP32 copies
    // regions: atom A uses region rid = reg_id[A]; its atoms are
    // reg_atoms[reg_off[rid] .. reg_off[rid] + reg_len[rid]) (ascending) and
    // its local block rows are lrp[lrp_off[rid] .. + reg_len[rid] + 1)
    // (absolute offsets into lblk, entries (local column atom, global block)).
    const int32_t *reg_id;
    const int64_t *reg_off;
    const int32_t *reg_len;
    const int64_t *lrp_off;
    const int64_t *lrp;
    const int2 *lblk;
    const int32_t *jloc;       // local position of atom A inside its region
    const int32_t *blk_loc;    // per global block: local position of its column atom
                               // inside the region of its row atom
    const int32_t *out_loc;    // n_atoms * kNbOut: local position (in the atom's own
                               // region) of its kNbOut nearest atoms, -1 if outside
    int max_nat;               // largest region (atoms)
    int max_lnnz;              // largest region operator (local blocks)
    int lidx;                  // 1: the workspace kernel can stage a region's local
                               // block index in LDS beside its other buffers
};

// One solve.  Columns are processed in chunks of the processing order: the
// basis kernel of a chunk writes, per column, the Galerkin pair and the
// basis rows the outputs need into a chunk buffer (`mid`), and the
// eigensolver kernel turns them into Ritz values, weights and amplitudes (or,
// with a given chemical potential, into rho, pi and E_j, N_j directly).
struct DevJob {
    int ncols;
    const int32_t *cols;       // global column per output row c
    const int32_t *order;      // processing order: order[idx] = c
    int p, q, nu;
    int precision;             // 0 FP64, 1 mixed (FP32 sums), 2 mixed (FP64 sums)
    double cg_tol, inner_tol, tau;
    int max_refine;
    int *queue;                // work counters, one per queue (reset before each chunk)
    int nqueues;               // 1, or 8 (one per XCD)
    const int32_t *qbounds;    // nqueues + 1 absolute offsets into order, this chunk
    int *fail;                 // [0] = first failing c (INT_MAX none)
    const int32_t *gstart;     // atom-group kernel: columns of group g are order positions
                               // gstart[g] .. gstart[g+1]
    int lidx;                  // 1: the basis kernel stages each region's local block
                               // index in LDS
    double *ws;                // basis workspace of the large-region kernel, slots * ws_stride
    int64_t ws_stride;
    // chunk: order positions c0 .. c0 + cn; slot s = position - c0
    int c0, cn;
    double *mid;               // cn * mid_stride doubles
    int64_t mid_stride;        // 2 nu^2 + (maxpat + 2) nu
    // per column outputs
    double *eps;               // ncols * nu
    double *wts;               // ncols * nu
    void *amp;                 // v_ia v_ja at the pattern rows (rank order): FP64 for
                               // precision 0, FP32 otherwise; column c starts at element
    const int64_t *amp_off;    // amp_off[c] and holds npat(c) * nu entries
    int32_t *stats;            // ncols * kStats
    const float *x0;           // optional: predicted s_j on the kNbOut nearest atoms
                               // (ncols * kNbOut * o), else zero start
    const double *x0full;      // optional: a start for s_j on the whole region (ncols *
                               // nmax, local order), e.g. the previous geometry's s_j
    double *sj_store;          // optional: s_j of global column j kept at j * nmax
    int32_t *sj_have;          // with sj_store: 1 where column j's s_j was kept
    float *sj_near;            // optional output: converged s_j on the same orbitals
    // Given chemical potential: the eigensolver kernel applies the Fermi
    // weights and writes rho, pi (either may be null) and E_j, N_j.
    int direct;
    double mu, kT;
    double *rho, *pi, *Ecol, *Ncol;
};

// Slot layout of the chunk buffer (doubles, row stride nu):
//   [0, nu^2)             X = U^T H U (at least its upper triangle; the
//                         eigensolver symmetrises)
//   [nu^2, 2 nu^2)        U^T S U
//   [2 nu^2, ...)         row 0: u_m at the local row of j, row 1: (S u_m) at
//                         that row, row 2 + t: u_m at pattern row t of j
inline int64_t mid_stride_of(int nu, int maxpat) { return 2 * (int64_t)nu * nu + (int64_t)(maxpat + 2) * nu; }

constexpr int kStats = 8;      // nu_eff, CG iterations, FP64 residual evaluations, status,
                               // start used (0 zero, 1 learned, 2 learned rejected), 3 spare

// Basis kernels.  Workspace kernel: one column per workgroup, U, S U, H U
// and the chain in a global workspace.  On-chip kernel: one column per
// workgroup, U in LDS and S U, chain in registers (regions of at most
// kSmallRows orbitals, nu <= 32, q <= nu_cap / 2).  Atom-group kernel: the
// requested columns of one atom in lockstep (o = 4 or 9), one SpMM per step
// for all of them, bases in the workspace.
constexpr int kMaxQueues = 8;
constexpr int kSmallRows = 512;
enum { kBasisWorkspace = 0, kBasisOnchip = 1, kBasisGroup = 2, kBasisAtom = 3 };
bool basis_small_fits(int nmax, int nu, int q, int o);
bool basis_group_fits(int nmax, int nu, int o);
// Atom kernel: the o columns of one atom in lockstep, every operator pass an
// SpMM over one staged set (o = 4 or 9; FP64 and FP64-accumulation modes).
bool basis_atom_fits(int nmax, int nu, int o, int precision);
bool atom_lidx_fits(int nmax, int o, int max_nat, int max_lnnz);
__host__ __device__ int64_t atom_slice_doubles(int nu, int q, int64_t ld);
__host__ __device__ int64_t atom_ws_doubles(int o, int nu, int q, int64_t ld);
int basis_group_width(int o);   // columns of one atom solved together
size_t basis_smem_bytes(int nmax, int nu, int kind, int o);
// whether the workspace (resp. on-chip) kernel keeps a region's local block
// index in LDS
bool global_lidx_fits(int nmax, int max_nat, int max_lnnz);
bool onchip_lidx_fits(int nmax, int nu, int max_nat, int max_lnnz);
int basis_rows_per_thread(int nmax);
hipError_t launch_reset(int *queue, int *fail, int reset_fail, hipStream_t st);
hipError_t launch_basis(const DevSystem &S, const DevJob &J, int kind, int slots, hipStream_t st);
hipError_t basis_occupancy(const DevSystem &S, const DevJob &J, int kind, int *blocks_per_cu);

// Batched reduced eigenproblems and column outputs, one wavefront per column
// of the chunk.
hipError_t launch_eig(const DevSystem &S, const DevJob &J, hipStream_t st);

// Fermi weighting, chemical potential, reductions.
hipError_t launch_minmax(const double *eps, const int32_t *stats, int ncols, int nu,
                         double kT, double *lohi, double *partial, hipStream_t st);
hipError_t launch_bisect(const double *eps, const double *wts, const int32_t *stats,
                         int ncols, int nu, double kT, double n_target, double *lohi,
                         double *partial, hipStream_t st);
hipError_t launch_rho(const DevSystem &S, const DevJob &J, const double *mu_ptr, double kT,
                      double *rho, double *pi, double *Ecol, double *Ncol, hipStream_t st);
hipError_t launch_sum2(const double *a, const double *b, int n, double *out, hipStream_t st);

// Forces, density of states and Green's function from a solve's outputs
// (ma_post.hip).
hipError_t launch_forces(int n_atoms, int o, const int64_t *blk_ptr, const int32_t *blk_col,
                         const int32_t *blk_t, const double *dH, const double *dS,
                         const double *rho, const double *pi, double spin, double *F,
                         hipStream_t st);
size_t dos_partial_doubles(int ncols, int nu, int nE);
hipError_t launch_dos(const double *eps, const double *wts, const int32_t *stats, int ncols,
                      int nu, const double *E, int nE, double eta, double spin, double *part,
                      double *out, hipStream_t st);
hipError_t launch_green(const DevSystem &S, const DevJob &J, double zr, double zi, double *gre,
                        double *gim, hipStream_t st);
// Map kept s_j (old regions) onto the current regions: x0full[c][i].
struct RegionView {
    const int32_t *reg_id, *reg_len, *reg_atoms;
    const int64_t *reg_off;
    int nmax;
};
hipError_t launch_map_sj(int ncols, const int32_t *cols, int o, RegionView cur, RegionView old,
                         const double *store, const int32_t *have, double *x0full, hipStream_t st);

// Allocation-free solve: a static device scratch of kScratchBytes per device
// (ma_noalloc.hip).  scratch_address returns this device's address of it; the
// device must be current.
constexpr size_t kScratchBytes = (size_t)256 << 20;
hipError_t scratch_address(int device, void **ptr, size_t *bytes);

// Start network (ma_mlp.hip).
hipError_t launch_features(const int32_t *cols, int ncols, int o, const float *geo, int nf_geo,
                           int nf, float *feat, hipStream_t st);
hipError_t launch_gather_rows(const float *in, const int32_t *idx, int64_t n, int m, int64_t rows,
                              float *out, int *bad, hipStream_t st);
hipError_t launch_to_bf16_t(const float *W, int rows, int cols, int rows_pad, int cols_pad,
                            unsigned short *Wt, hipStream_t st);
size_t mlp_infer_smem(int nf_pad, int nh);
hipError_t launch_mlp_infer(const float *X, int64_t n, int nf, int nf_pad, int nh, int no,
                            const unsigned short *W1t, const float *b1, const unsigned short *W2t,
                            const float *b2, const unsigned short *W3t, const float *b3, float *Y,
                            hipStream_t st);
hipError_t launch_gemm(int M, int N, int K, const float *A, int64_t sa0, int64_t sa1,
                       const int32_t *gather, const float *B, int64_t sb0, int64_t sb1,
                       const float *bias, float beta, float *C, int64_t ldc, float *Z, hipStream_t st);
hipError_t launch_mse(const float *Y, const float *T, const int32_t *gather, int64_t n, int no,
                      float *dY, double *partial, int nblocks, hipStream_t st);
hipError_t launch_silu_bwd(float *G, const float *Z, int64_t total, hipStream_t st);
hipError_t launch_colsum(const float *G, int64_t n, int m, float *db, hipStream_t st);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t count, float lr,
                       float b1, float b2, float eps, int step, hipStream_t st);

}  // namespace ma
