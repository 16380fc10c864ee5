// Internal declarations shared by the host side (ma_host.cpp) and the
// kernels (ma_kernels.hip) of libmarnoldi.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ma {

constexpr int kThreads = 256;            // workgroup size of the column kernel
constexpr int kWaves = kThreads / 64;
constexpr int kMaxNu = 64;
constexpr int kBisectTrials = 63;        // trial potentials per bisection pass
constexpr int kBisectPasses = 9;         // 64^9 narrows any bracket below 1e-15
constexpr int kCountBlocks = 256;        // fixed grid of the electron-count kernel
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
};

// One solve.
struct DevJob {
    int ncols;
    const int32_t *cols;       // global column per output row c
    const int32_t *order;      // processing order (LPT): order[idx] = c
    int p, q, nu;
    int precision;             // 0 FP64, 1 mixed
    double cg_tol, inner_tol, tau;
    int max_refine;
    int *queue;                // work counters, one per queue (reset before launch)
    int nqueues;               // 1, or 8 (one per XCD)
    const int32_t *qbounds;    // nqueues + 1 offsets into order
    int *fail;                 // [0] = first failing c (INT_MAX none)
    double *ws;                // workspace, slots * ws_stride doubles
    int64_t ws_stride;
    // per column outputs
    double *eps;               // ncols * nu
    double *wts;               // ncols * nu
    double *amp;               // ncols * maxpat * nu: v_ia v_ja at pattern rows
    int32_t *stats;            // ncols * kStats
    const float *x0;           // optional: predicted s_j on the kNbOut nearest atoms
                               // (ncols * kNbOut * o), else zero start
    float *sj_near;            // optional output: converged s_j on the same orbitals
};

constexpr int kStats = 8;      // nu_eff, CG iterations, FP64 residual evaluations, status,
                               // start used (0 zero, 1 learned, 2 learned rejected), 3 spare

// Shared-memory bytes the column kernel needs.
size_t solve_smem_bytes(int nmax, int nu);

// Launchers (all asynchronous on `st`).
constexpr int kMaxQueues = 8;
hipError_t launch_reset(int *queue, int *fail, hipStream_t st);
hipError_t launch_solve(const DevSystem &S, const DevJob &J, int slots, hipStream_t st);
int solve_rows_per_thread(int nmax);
hipError_t solve_occupancy(const DevSystem &S, const DevJob &J, int *blocks_per_cu);

// Fermi weighting, chemical potential, reductions.
hipError_t launch_minmax(const double *eps, const int32_t *stats, int ncols, int nu,
                         double kT, double *lohi, hipStream_t st);
hipError_t launch_bisect(const double *eps, const double *wts, const int32_t *stats,
                         int ncols, int nu, double kT, double n_target, double *lohi,
                         double *partial, hipStream_t st);
hipError_t launch_rho(const DevSystem &S, const DevJob &J, const double *mu_ptr, double mu,
                      double kT, double *rho, double *pi, double *Ecol, double *Ncol,
                      hipStream_t st);
hipError_t launch_sum2(const double *a, const double *b, int n, double *out, hipStream_t st);

// Start network (ma_mlp.hip).
hipError_t launch_features(const int32_t *cols, int ncols, int o, const float *geo, int nf_geo,
                           int nf, float *feat, hipStream_t st);
hipError_t launch_gather_rows(const float *in, const int32_t *idx, int64_t n, int m, float *out,
                              hipStream_t st);
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
