// Quantities built from the column outputs of a solve (gfx950):
//
//   forces   F_K = -spin sum_j sum_i [rho_ij dH_ji/dR_K - pi_ij dS_ji/dR_K]
//            (Sec. 2: the force as a sum of partial sums over the columns j;
//            only pattern elements enter, and the derivative blocks are
//            nonzero only between neighbouring atoms)
//   DOS      D(E) = spin/pi sum_j sum_a w_a eta / ((E - eps_a)^2 + eta^2),
//            the S-weighted trace of the subspace Green's functions at
//            E + i eta (Eqs. 11-12), from the Ritz values and weights
//   G(z)     G_ij(z) = sum_a v_ia v_ja / (z - eps_a) at the pattern
//            elements (Eq. 12 applied to e_j, Eq. 11), from the stored
//            amplitudes v_ia v_ja of a solve that bisected mu
//
// All reductions run in a fixed order: results are bitwise reproducible.
#include "ma_device.h"

namespace ma {

namespace {

// One wavefront per atom X (persistent over the atoms):
// F_X = spin sum over blocks k = (X, B), B != X, of g_k - g_T(k), where
// g_k = sum_{r,c} rho_k[r][c] dH_k[:][r][c] - pi_k[r][c] dS_k[:][r][c] and
// T(k) is the block (B, X).  Block k = (A, B) holds columns j = (A, r) at
// rows i = (B, c); dH_k is the derivative of H_AB with respect to R_B, so
// g_k enters F_A with + and F_B with -.
__global__ void __launch_bounds__(64) k_forces(int n_atoms, int o, const int64_t *blk_ptr,
                                               const int32_t *blk_col, const int32_t *blk_t,
                                               const double *dH, const double *dS,
                                               const double *rho, const double *pi, double spin,
                                               double *F)
{
    const int lane = threadIdx.x;
    const int oo = o * o;
    for (int X = blockIdx.x; X < n_atoms; X += gridDim.x) {
        double f0 = 0.0, f1 = 0.0, f2 = 0.0;
        for (int64_t k = blk_ptr[X]; k < blk_ptr[X + 1]; ++k) {
            if (blk_col[k] == X) continue;
            const int64_t kt = blk_t[k];
            for (int e = lane; e < oo; e += 64) {
                const double ra = rho[k * oo + e], pa = pi[k * oo + e];
                const double rb = rho[kt * oo + e], pb = pi[kt * oo + e];
                const double *ha = dH + k * 3 * oo + e, *sa = dS + k * 3 * oo + e;
                const double *hb = dH + kt * 3 * oo + e, *sb = dS + kt * 3 * oo + e;
                f0 += (ra * ha[0] - pa * sa[0]) - (rb * hb[0] - pb * sb[0]);
                f1 += (ra * ha[oo] - pa * sa[oo]) - (rb * hb[oo] - pb * sb[oo]);
                f2 += (ra * ha[2 * oo] - pa * sa[2 * oo]) - (rb * hb[2 * oo] - pb * sb[2 * oo]);
            }
        }
        f0 = wave_sum(f0);
        f1 = wave_sum(f1);
        f2 = wave_sum(f2);
        if (lane == 0) {
            F[3 * (int64_t)X] = spin * f0;
            F[3 * (int64_t)X + 1] = spin * f1;
            F[3 * (int64_t)X + 2] = spin * f2;
        }
    }
}

constexpr int kDosChunk = 8192;   // Ritz pairs per workgroup of the DOS kernel
constexpr int kDosTile = 256;     // energies per workgroup

// Partial DOS of one chunk of Ritz pairs (staged in LDS) at a tile of
// energies: part[chunk][E] (thread t takes energy tile * 256 + t).
__global__ void __launch_bounds__(256) k_dos_part(const double *eps, const double *wts,
                                                  const int32_t *stats, int ncols, int nu,
                                                  const double *E, int nE, double eta,
                                                  double *part)
{
    __shared__ double se[kDosChunk / 4], sw[kDosChunk / 4];
    const int64_t npairs = (int64_t)ncols * nu;
    const int64_t p0 = (int64_t)blockIdx.x * kDosChunk;
    const int ie = blockIdx.y * kDosTile + threadIdx.x;
    const double en = ie < nE ? E[ie] : 0.0;
    double acc = 0.0;
    for (int64_t s0 = p0; s0 < p0 + kDosChunk && s0 < npairs; s0 += kDosChunk / 4) {
        const int cnt = (int)min<int64_t>(kDosChunk / 4, min<int64_t>(npairs, p0 + kDosChunk) - s0);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += 256) {
            const int64_t g = s0 + t;
            const int c = (int)(g / nu), a = (int)(g - (int64_t)c * nu);
            const bool ok = a < stats[(int64_t)c * kStats];
            se[t] = ok ? eps[g] : 0.0;
            sw[t] = ok ? wts[g] : 0.0;
        }
        __syncthreads();
        for (int t = 0; t < cnt; ++t) {
            const double d = en - se[t];
            acc += sw[t] * eta / (d * d + eta * eta);
        }
    }
    if (ie < nE) part[(int64_t)blockIdx.x * nE + ie] = acc;
}

// D(E) = spin / pi * sum over chunks (fixed order)
__global__ void __launch_bounds__(256) k_dos_sum(const double *part, int nchunks, int nE,
                                                 double spin, double *out)
{
    const int ie = blockIdx.x * 256 + threadIdx.x;
    if (ie >= nE) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * nE + ie];
    out[ie] = spin / M_PI * s;
}

// G_ij(z) at the pattern slots of every solved column from the stored
// amplitudes (TA: FP64 or FP32), one workgroup per column.
template <typename TA>
__global__ void __launch_bounds__(128) k_green(DevSystem S, DevJob J, double zr, double zi,
                                               double *gre, double *gim)
{
    __shared__ double cr[kMaxNu], ci[kMaxNu];
    const int o = S.o, nu = J.nu;
    for (int c = blockIdx.x; c < J.ncols; c += gridDim.x) {
        const int j = J.cols[c];
        const int A = j / o, r = j - A * o;
        const int L = J.stats[(int64_t)c * kStats];
        __syncthreads();
        for (int a = threadIdx.x; a < nu; a += blockDim.x) {
            // 1 / (z - eps) = conj(z - eps) / |z - eps|^2
            const double dr = zr - J.eps[(int64_t)c * nu + a], di = zi;
            const double den = dr * dr + di * di;
            cr[a] = a < L ? dr / den : 0.0;
            ci[a] = a < L ? -di / den : 0.0;
        }
        __syncthreads();
        const int64_t kb0 = S.blk_ptr[A];
        const int npat = (int)(S.blk_ptr[A + 1] - kb0) * o;
        const TA *amp = reinterpret_cast<const TA *>(J.amp) + J.amp_off[c];
        for (int t = threadIdx.x; t < npat; t += blockDim.x) {
            double sr = 0.0, si = 0.0;
            for (int a = 0; a < L; ++a) {
                const double am = (double)amp[t * nu + a];
                sr += cr[a] * am;
                si += ci[a] * am;
            }
            const int64_t slot = ((kb0 + t / o) * o + r) * o + (t % o);
            if (gre) gre[slot] = sr;
            if (gim) gim[slot] = si;
        }
    }
}

// Start vectors from kept s_j: for column c (global j, atom A), row i of
// the current region of A (atom b = its i / o-th atom) takes the kept value
// of the same orbital of b in A's region at the time of keeping, or zero if b
// was not in it (both atom lists ascending: binary search).
__global__ void __launch_bounds__(128) k_map_sj(int ncols, const int32_t *cols, int o,
                                                RegionView cur, RegionView old,
                                                const double *store, const int32_t *have,
                                                double *x0full)
{
    for (int c = blockIdx.x; c < ncols; c += gridDim.x) {
        const int j = cols[c];
        const int A = j / o;
        const int rid = cur.reg_id[A], orid = old.reg_id[A];
        const int32_t *ca = cur.reg_atoms + cur.reg_off[rid];
        const int32_t *oa = old.reg_atoms + old.reg_off[orid];
        const int len = cur.reg_len[rid], olen = old.reg_len[orid];
        const bool kept = have[j] != 0;
        const double *src = store + (int64_t)j * old.nmax;
        double *dst = x0full + (int64_t)c * cur.nmax;
        for (int t = threadIdx.x; t < len; t += blockDim.x) {
            const int b = ca[t];
            int lo = 0, hi = olen;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (oa[mid] < b) lo = mid + 1;
                else hi = mid;
            }
            const bool found = kept && lo < olen && oa[lo] == b;
            for (int r = 0; r < o; ++r) dst[t * o + r] = found ? src[lo * o + r] : 0.0;
        }
    }
}

}  // namespace

hipError_t launch_map_sj(int ncols, const int32_t *cols, int o, RegionView cur, RegionView old,
                         const double *store, const int32_t *have, double *x0full, hipStream_t st)
{
    const int grid = ncols < 65536 ? ncols : 65536;
    hipLaunchKernelGGL(k_map_sj, dim3(grid), dim3(128), 0, st, ncols, cols, o, cur, old, store,
                       have, x0full);
    return hipGetLastError();
}

hipError_t launch_forces(int n_atoms, int o, const int64_t *blk_ptr, const int32_t *blk_col,
                         const int32_t *blk_t, const double *dH, const double *dS,
                         const double *rho, const double *pi, double spin, double *F,
                         hipStream_t st)
{
    const int grid = n_atoms < (1 << 20) ? n_atoms : (1 << 20);
    hipLaunchKernelGGL(k_forces, dim3(grid), dim3(64), 0, st, n_atoms, o, blk_ptr, blk_col, blk_t,
                       dH, dS, rho, pi, spin, F);
    return hipGetLastError();
}

size_t dos_partial_doubles(int ncols, int nu, int nE)
{
    const int64_t npairs = (int64_t)ncols * nu;
    const int64_t nchunks = (npairs + kDosChunk - 1) / kDosChunk;
    return (size_t)nchunks * nE;
}

hipError_t launch_dos(const double *eps, const double *wts, const int32_t *stats, int ncols,
                      int nu, const double *E, int nE, double eta, double spin, double *part,
                      double *out, hipStream_t st)
{
    const int64_t npairs = (int64_t)ncols * nu;
    const int nchunks = (int)((npairs + kDosChunk - 1) / kDosChunk);
    const int tiles = (nE + kDosTile - 1) / kDosTile;
    if (nchunks < 1 || tiles < 1) return hipSuccess;
    hipLaunchKernelGGL(k_dos_part, dim3(nchunks, tiles), dim3(256), 0, st, eps, wts, stats, ncols,
                       nu, E, nE, eta, part);
    hipLaunchKernelGGL(k_dos_sum, dim3(tiles), dim3(256), 0, st, part, nchunks, nE, spin, out);
    return hipGetLastError();
}

hipError_t launch_green(const DevSystem &S, const DevJob &J, double zr, double zi, double *gre,
                        double *gim, hipStream_t st)
{
    const int grid = J.ncols < 65536 ? J.ncols : 65536;
    if (J.precision == 0)
        hipLaunchKernelGGL(k_green<double>, dim3(grid), dim3(128), 0, st, S, J, zr, zi, gre, gim);
    else
        hipLaunchKernelGGL(k_green<float>, dim3(grid), dim3(128), 0, st, S, J, zr, zi, gre, gim);
    return hipGetLastError();
}

}  // namespace ma
