// Launchers of libmarnoldi's kernels (gfx950).  The kernels themselves are
// in ma_device.h; the basis-kernel families are instantiated in the
// ma_basis_*.hip files, which hand their host stubs to the dispatch below.
#include "ma_device.h"

namespace ma {

namespace {

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
template <typename K>
hipError_t launch_with_smem(K kern, int grid, int block, size_t smem, hipStream_t st,
                            const DevSystem &S, const DevJob &J)
{
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    DevSystem s_arg = S;
    DevJob j_arg = J;
    void *args[] = {&s_arg, &j_arg};
    return hipLaunchKernel((const void *)kern, dim3(grid), dim3(block), args, smem, st);
}

template <typename K>
hipError_t occupancy_of(K kern, int block, size_t smem, int *bpc)
{
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(bpc, kern, block, smem);
}

int small_threads(int nmax) { return nmax <= 256 ? 256 : 512; }
int small_nu_cap(int nu) { return nu <= 16 ? 16 : 32; }

void *small_kernel(int o, int nt, int nucap, int prec) { return basis_s_kernel(o, nt, nucap, prec); }

void *global_kernel(int o, int R, int prec)
{
    if (o == 4) return basis_g_kernel_o4(R, prec);
    if (o == 9) return basis_g_kernel_o9(R, prec);
    return basis_g_kernel_o0(R, prec);
}

typedef void (*basis_fn)(DevSystem, DevJob);

void *group_kernel(int o, int nmax, int prec)
{
    (void)nmax;
    return basis_m_kernel(o, prec);
}

}  // namespace

int basis_group_width(int o) { return o == 9 ? 3 : o == 4 ? 4 : 0; }

// LDS of the atom kernel besides the region index: one staged set of o
// vectors (FP64) and the fixed shared state (column states, dot-sweep jobs,
// reduction scratch; 8 KB bounds it)
size_t atom_smem_bytes(int nmax, int o) { return sizeof(double) * (size_t)nmax * o; }
constexpr size_t kAtomStaticLds = 8 * 1024;

bool basis_atom_fits(int nmax, int nu, int o, int precision)
{
    (void)nu;
    if (!(o == 4 || o == 9) || precision == 1) return false;
    return atom_smem_bytes(nmax, o) + kAtomStaticLds <= 160 * 1024;
}

bool basis_group_fits(int nmax, int nu, int o)
{
    if (!((o == 4 && nmax <= 512) || (o == 9 && nmax <= 1024))) return false;
    return basis_smem_bytes(nmax, nu, kBasisGroup, o) <= 160 * 1024;
}

bool basis_small_fits(int nmax, int nu, int q, int o)
{
    (void)o;
    if (nmax > kSmallRows || nu > 32) return false;
    const int nucap = small_nu_cap(nu);
    if (q > nucap / 2) return false;
    return basis_smem_bytes(nmax, nu, kBasisOnchip, o) <= 160 * 1024;
}

int basis_rows_per_thread(int nmax)
{
    const int r = (nmax + NTG - 1) / NTG;
    if (r <= 4) return r < 1 ? 1 : r;
    if (r <= 6) return 6;
    return 8;
}

// LDS of a staged region block index
size_t lidx_bytes(int max_nat, int max_lnnz)
{
    return sizeof(int) * (size_t)((max_nat + 2) & ~1) + sizeof(int2) * (size_t)max_lnnz;
}

bool onchip_lidx_fits(int nmax, int nu, int max_nat, int max_lnnz)
{
    return basis_smem_bytes(nmax, nu, kBasisOnchip, 0) + lidx_bytes(max_nat, max_lnnz) <= 160 * 1024;
}

// whether the atom kernel keeps the region index in LDS: only where two
// workgroups still fit on a compute unit
bool atom_lidx_fits(int nmax, int o, int max_nat, int max_lnnz)
{
    return atom_smem_bytes(nmax, o) + lidx_bytes(max_nat, max_lnnz) + kAtomStaticLds <= 80 * 1024;
}

bool global_lidx_fits(int nmax, int max_nat, int max_lnnz)
{
    return sizeof(double) * (size_t)global_smem_doubles(nmax) + lidx_bytes(max_nat, max_lnnz) <=
           80 * 1024;
}

size_t basis_smem_bytes(int nmax, int nu, int kind, int o)
{
    if (kind == kBasisOnchip) {
        const int nt = small_threads(nmax), nucap = small_nu_cap(nu);
        const int fixed = nt == 256 ? (nucap == 16 ? small_smem_doubles_fixed<256, 16>()
                                                   : small_smem_doubles_fixed<256, 32>())
                                    : (nucap == 16 ? small_smem_doubles_fixed<512, 16>()
                                                   : small_smem_doubles_fixed<512, 32>());
        return sizeof(double) * ((size_t)nu * nmax + 3 * (size_t)nmax + fixed);
    }
    if (kind == kBasisAtom) return atom_smem_bytes(nmax, o);
    if (kind == kBasisGroup) {
        const int b = basis_group_width(o);
        return sizeof(double) * (2 * (size_t)b * nmax + 2 * (size_t)b * kMaxNu + (512 / 64) * 16);
    }
    return sizeof(double) * (size_t)global_smem_doubles(nmax);
}

hipError_t launch_reset(int *queue, int *fail, int reset_fail, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, st, queue, fail, reset_fail);
    return hipGetLastError();
}

hipError_t launch_basis(const DevSystem &S, const DevJob &J, int kind, int slots, hipStream_t st)
{
    const size_t smem = basis_smem_bytes(S.nmax, J.nu, kind, S.o) +
                        (J.lidx ? lidx_bytes(S.max_nat, S.max_lnnz) : 0);
    if (kind == kBasisOnchip) {
        const int nt = small_threads(S.nmax);
        basis_fn k = (basis_fn)small_kernel(S.o, nt, small_nu_cap(J.nu), J.precision);
        return launch_with_smem(k, slots, nt, smem, st, S, J);
    }
    if (kind == kBasisGroup) {
        basis_fn k = (basis_fn)group_kernel(S.o, S.nmax, J.precision);
        return launch_with_smem(k, slots, 512, smem, st, S, J);
    }
    if (kind == kBasisAtom) {
        basis_fn k = (basis_fn)basis_a_kernel(S.o, basis_rows_per_thread(S.nmax), J.precision);
        return launch_with_smem(k, slots, 256, smem, st, S, J);
    }
    basis_fn k = (basis_fn)global_kernel(S.o, basis_rows_per_thread(S.nmax), J.precision);
    return launch_with_smem(k, slots, NTG, smem, st, S, J);
}

hipError_t basis_occupancy(const DevSystem &S, const DevJob &J, int kind, int *bpc)
{
    const size_t smem = basis_smem_bytes(S.nmax, J.nu, kind, S.o) +
                        (J.lidx ? lidx_bytes(S.max_nat, S.max_lnnz) : 0);
    if (kind == kBasisOnchip) {
        const int nt = small_threads(S.nmax);
        return occupancy_of((basis_fn)small_kernel(S.o, nt, small_nu_cap(J.nu), J.precision), nt,
                            smem, bpc);
    }
    if (kind == kBasisGroup)
        return occupancy_of((basis_fn)group_kernel(S.o, S.nmax, J.precision), 512, smem, bpc);
    if (kind == kBasisAtom)
        return occupancy_of((basis_fn)basis_a_kernel(S.o, basis_rows_per_thread(S.nmax), J.precision),
                            256, smem, bpc);
    return occupancy_of((basis_fn)global_kernel(S.o, basis_rows_per_thread(S.nmax), J.precision),
                        NTG, smem, bpc);
}

hipError_t launch_eig(const DevSystem &S, const DevJob &J, hipStream_t st)
{
    const size_t smem = sizeof(double) * (2 * (size_t)J.nu * J.nu + 10 * (size_t)J.nu) +
                        sizeof(int) * 2 * (size_t)J.nu;
    const int grid = J.cn < (1 << 20) ? J.cn : (1 << 20);
    if (grid < 1) return hipSuccess;
    if (J.precision == 0) return launch_with_smem(k_eig<double>, grid, 64, smem, st, S, J);
    return launch_with_smem(k_eig<float>, grid, 64, smem, st, S, J);
}

// grid of the bracket and count kernels: about 2,048 Ritz pairs per
// workgroup, between 64 and kCountBlocks workgroups
int count_grid(int ncols, int nu)
{
    const int64_t g = ((int64_t)ncols * nu + 2047) / 2048;
    return g < 64 ? 64 : g > kCountBlocks ? kCountBlocks : (int)g;
}

hipError_t launch_minmax(const double *eps, const int32_t *stats, int ncols, int nu, double kT,
                         double *lohi, double *partial, hipStream_t st)
{
    const int grid = count_grid(ncols, nu);
    hipLaunchKernelGGL(k_minmax, dim3(grid), dim3(256), 0, st, eps, stats, ncols, nu, partial);
    hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(64), 0, st, partial, grid, kT, lohi,
                       count_done(partial));
    return hipGetLastError();
}

hipError_t launch_bisect(const double *eps, const double *wts, const int32_t *stats, int ncols,
                         int nu, double kT, double n_target, double *lohi, double *partial,
                         hipStream_t st)
{
    const int grid = count_grid(ncols, nu);
    for (int pass = 0; pass < kBisectPasses; ++pass)
        hipLaunchKernelGGL(k_count, dim3(grid), dim3(256), 0, st, eps, wts, stats, ncols, nu, kT,
                           n_target, lohi, partial, count_done(partial));
    return hipGetLastError();
}

hipError_t launch_rho(const DevSystem &S, const DevJob &J, const double *mu_ptr, double kT,
                      double *rho, double *pi, double *Ecol, double *Ncol, hipStream_t st)
{
    const int grid = J.ncols < 65536 ? J.ncols : 65536;
    const size_t blk = (size_t)S.maxpat * J.nu * (J.precision == 0 ? sizeof(double) : sizeof(float));
    const int stage = blk <= 48 * 1024 ? 1 : 0;
    const size_t smem = stage ? blk : 0;
    if (J.precision == 0)
        hipLaunchKernelGGL(k_rho<double>, dim3(grid), dim3(128), smem, st, S, J, mu_ptr, kT, rho,
                           pi, Ecol, Ncol, stage);
    else
        hipLaunchKernelGGL(k_rho<float>, dim3(grid), dim3(128), smem, st, S, J, mu_ptr, kT, rho,
                           pi, Ecol, Ncol, stage);
    return hipGetLastError();
}

hipError_t launch_sum2(const double *a, const double *b, int n, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum2, dim3(1), dim3(1024), 0, st, a, b, n, out);
    return hipGetLastError();
}

}  // namespace ma

