// Device code of libmarnoldi (gfx950): the kernels and their helpers.
// Included by ma_kernels.hip (launchers) and by the ma_basis_*.hip files,
// each of which instantiates one family of basis kernels, so that the
// families compile in parallel.  Everything here has internal linkage.
#pragma once

// Device kernels of libmarnoldi (gfx950).
//
// The per-column multiple Arnoldi solve (arXiv:1202.0098, Sec. 2) runs as two
// kernels per chunk of columns.
//
// Basis kernel (persistent workgroups draining work queues), per column:
//   inner CG for s_j = S_A^-1 e_j                 (Sec. 2, inner CG loop)
//   S-orthonormal basis of K_p(H;e_j)+K_q(H;s_j)  (Eqs. 4, 6-9)
//   Galerkin pair X = U^T H U, S~ = U^T S U        (Sec. 2, Galerkin principle)
// H_A, S_A are the principal submatrices of H, S on the region of atom(j)
// (real-space projection, Sec. 3), read through a per-region local block
// index.  Thread t owns local rows t, t + NT, ...; the vector an SpMV reads
// is staged in LDS.  Three variants:
//   k_basis_s  regions of at most 512 orbitals, nu <= 32: U lives in LDS,
//              S U and the block-2 chain in registers (row-owned), and the
//              Galerkin pair is accumulated as each vector is accepted, so the
//              basis never leaves the compute unit;
//   k_basis_g  any region: U, S U, H U and the chain live in a per-workgroup
//              slice of a global workspace, the second Gram-Schmidt pass of
//              each vector is delayed into the next step (one dot sweep and
//              one update sweep per vector) and the pair is formed on the
//              FP64 matrix cores;
//   k_basis_m  the columns of one atom in lockstep, every SpMV an SpMM.
// All write the pair and the basis rows the outputs need into a chunk buffer.
//
// Eigensolver kernel (one wavefront per column): Cholesky of S~, Householder
// tridiagonalisation and implicit QL of L^-1 H~ L^-T, the Ritz vectors at
// the rows of the outputs, Ritz values and weights, and either the
// amplitudes v_ia v_ja (chemical potential still to be found) or the
// Fermi-weighted rho, pi, E_j, N_j (Eqs. 13-14, 17).
//
// The remaining kernels bisect the chemical potential on the electron count
// (Sec. 2, summation over j), weight the stored amplitudes with the Fermi
// function and reduce the column energies in a fixed order.
#include <float.h>
#include <limits.h>
#include <math.h>

#include <type_traits>

#include "ma_internal.h"

namespace ma {

namespace {

constexpr int NTG = 256;           // workgroup size of the large-region kernel
constexpr int NWG = NTG / 64;

// ------------------------------------------------------------------------
// reductions (fixed order: results are bitwise reproducible)
// ------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the workgroup (NWV wavefronts).  Ends with a barrier, so the
// caller may overwrite shared buffers read before the call.
template <int NWV, typename T>
__device__ __forceinline__ T block_sum(T v, T *red)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    T s = 0;
#pragma unroll
    for (int k = 0; k < NWV; ++k) s += red[k];
    __syncthreads();
    return s;
}

// Transposed wavefront reduction of NV values per lane (NV a power of two,
// at most 32): log2(NV) halving exchanges, each lane keeping the half its
// lane bit selects, then a butterfly over the remaining lane bits.  Costs
// NV - 1 + 6 - log2(NV) exchanges instead of 6 NV.  Afterwards v[0] of lane l
// holds the wavefront total of value tr_index<NV>(l).
template <int NV>
__host__ __device__ constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2<NV>(v / 2); }

template <int NV>
__device__ __forceinline__ void wave_transpose_reduce(double (&v)[NV])
{
    constexpr int LG = ilog2<NV>(NV);
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int step = 0; step < LG; ++step) {
        const int half = NV >> (step + 1), off = 32 >> step;
        const bool hi = (lane & off) != 0;
#pragma unroll
        for (int k = 0; k < half; ++k) {
            const double lo_v = v[k], hi_v = v[k + half];
            const double send = hi ? lo_v : hi_v;
            const double keep = hi ? hi_v : lo_v;
            v[k] = keep + __shfl_xor(send, off, 64);
        }
    }
#pragma unroll
    for (int step = LG; step < 6; ++step) v[0] += __shfl_xor(v[0], 32 >> step, 64);
}

template <int NV>
__device__ __forceinline__ int tr_index(int lane)
{
    constexpr int LG = ilog2<NV>(NV);
    int idx = 0;
#pragma unroll
    for (int step = 0; step < LG; ++step)
        if (lane & (32 >> step)) idx += NV >> (step + 1);
    return idx;
}

// the lanes whose butterfly bits are zero hold every value exactly once
template <int NV>
__device__ __forceinline__ bool tr_writer(int lane) { return (lane & (64 / NV - 1)) == 0; }

// G groups of NV values per thread, summed over the workgroup: out[g*NV + k]
// (LDS) receives the total of value k of group g.  `gen(g, v)` fills group g;
// groups are produced and reduced one at a time to bound register use.
// Starts and ends with the scratch area free; ends with a barrier.
template <int NWV, int NV, int G, typename F>
__device__ __forceinline__ void block_reduce(F &&gen, double *scratch, double *out)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double res[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        double v[NV];
        gen(g, v);
        wave_transpose_reduce<NV>(v);
        res[g] = v[0];
    }
    if (tr_writer<NV>(lane)) {
        const int k = tr_index<NV>(lane);
#pragma unroll
        for (int g = 0; g < G; ++g) scratch[(w * G + g) * NV + k] = res[g];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < G * NV; t += NWV * 64) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NWV; ++k) s += scratch[k * G * NV + t];
        out[t] = s;
    }
    __syncthreads();
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Order the LDS traffic of one wavefront (its lanes execute together; LDS
// operations of a wavefront complete in issue order).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double fermi(double x)
{
    if (x <= 0.0) return 1.0 / (1.0 + exp(x));
    double e = exp(-x);
    return e / (1.0 + e);
}

// ------------------------------------------------------------------------
// column context
// ------------------------------------------------------------------------
struct Col {
    int n;               // local dimension
    int n_at;            // region atoms
    const int64_t *rp;   // local block-row pointers (n_at + 1)
    int jl;              // local index of j
    int A, r;            // atom and orbital of j
    bool lidx;           // the block index below is staged in LDS
    const int *srp;      // LDS: block-row pointers relative to rp[0]
    const int2 *sblk;    // LDS: the region's local blocks
};

__device__ __forceinline__ Col make_col(const DevSystem &S, const DevJob &J, int c, int o)
{
    Col g;
    const int j = J.cols[c];
    g.A = j / o;
    g.r = j - g.A * o;
    const int rid = S.reg_id[g.A];
    g.n_at = S.reg_len[rid];
    g.n = g.n_at * o;
    g.rp = S.lrp + S.lrp_off[rid];
    g.jl = S.jloc[g.A] * o + g.r;
    g.lidx = false;
    g.srp = nullptr;
    g.sblk = nullptr;
    return g;
}

// Copy the column's region block index into LDS (the whole workgroup), so
// every SpMV of the column reads it from there: one global round trip per
// SpMV (the operator values) instead of three dependent ones.
template <int NT>
__device__ __forceinline__ void stage_col_index(const DevSystem &S, Col &g, int *srp, int2 *sblk)
{
    const int64_t b0 = g.rp[0];
    const int nnz = (int)(g.rp[g.n_at] - b0);
    for (int a = threadIdx.x; a <= g.n_at; a += NT) srp[a] = (int)(g.rp[a] - b0);
    for (int k = threadIdx.x; k < nnz; k += NT) sblk[k] = S.lblk[b0 + k];
    __syncthreads();
    g.lidx = true;
    g.srp = srp;
    g.sblk = sblk;
}

// SpMV on the thread's own rows: hy = H x, sy = S x (x in LDS), zy = H xb.
// TM: stored operator values; TX: vector entries and accumulation.
template <int O, int R, int NT, typename TM, typename TX, bool DO_H, bool DO_S, bool DO_Z>
__device__ __forceinline__ void spmv_rows(const DevSystem &S, const Col &g, int o_rt,
                                          const TM *__restrict__ Hv, const TM *__restrict__ Sv,
                                          const TX *xa, const TX *xb, double (&hy)[R],
                                          double (&sy)[R], double (&zy)[R])
{
    const int o = O ? O : o_rt;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
        const int i = threadIdx.x + rr * NT;
        TX h = 0, s = 0, z = 0;
        if (i < g.n) {
            const int a = i / o;
            const int ri = i - a * o;
            auto blk = [&](const int2 e) __attribute__((always_inline)) {
                const int64_t base = (int64_t)e.y * (o * o) + ri * o;
                const int xo = e.x * o;
                if constexpr (O > 0) {
#pragma unroll
                    for (int cc = 0; cc < O; ++cc) {
                        const TX xv = xa[xo + cc];
                        if (DO_H) h += (TX)Hv[base + cc] * xv;
                        if (DO_S) s += (TX)Sv[base + cc] * xv;
                        if (DO_Z) z += (TX)Hv[base + cc] * xb[xo + cc];
                    }
                } else {
                    for (int cc = 0; cc < o; ++cc) {
                        const TX xv = xa[xo + cc];
                        if (DO_H) h += (TX)Hv[base + cc] * xv;
                        if (DO_S) s += (TX)Sv[base + cc] * xv;
                        if (DO_Z) z += (TX)Hv[base + cc] * xb[xo + cc];
                    }
                }
            };
            if (g.lidx) {
                const int k0 = g.srp[a], k1 = g.srp[a + 1];
                if constexpr (O == 0) {
                    for (int kb = k0; kb < k1; ++kb) blk(g.sblk[kb]);
                } else {
                    // batches of NB blocks whose value loads are issued
                    // before any product (blocks past the row's end read its
                    // first block and add nothing): more loads in flight per
                    // round trip than the unrolled loop gets (6 blocks: the
                    // spd cell's step 9 % faster)
                    constexpr int OB = O > 0 ? O : 1;
                    constexpr int NB = 6;
                    for (int kb = k0; kb < k1; kb += NB) {
                        int2 e[NB];
                        TM hm[NB][OB], sm[NB][OB];
#pragma unroll
                        for (int j = 0; j < NB; ++j) {
                            e[j] = g.sblk[kb + j < k1 ? kb + j : k0];
                            const int64_t base = (int64_t)e[j].y * (o * o) + ri * o;
#pragma unroll
                            for (int cc = 0; cc < OB; ++cc) {
                                if (DO_H || DO_Z) hm[j][cc] = Hv[base + cc];
                                if (DO_S) sm[j][cc] = Sv[base + cc];
                            }
                        }
#pragma unroll
                        for (int j = 0; j < NB; ++j) {
                            const bool ok = kb + j < k1;
                            const int xo = e[j].x * o;
#pragma unroll
                            for (int cc = 0; cc < OB; ++cc) {
                                const TX xv = xa[xo + cc];
                                if (DO_H) h += (ok ? (TX)hm[j][cc] : (TX)0) * xv;
                                if (DO_S) s += (ok ? (TX)sm[j][cc] : (TX)0) * xv;
                                if (DO_Z) z += (ok ? (TX)hm[j][cc] : (TX)0) * xb[xo + cc];
                            }
                        }
                    }
                }
            } else {
                // several blocks in flight: the index and value loads of a
                // block do not depend on the previous block
                const int64_t k0 = g.rp[a], k1 = g.rp[a + 1];
#pragma unroll 4
                for (int64_t kb = k0; kb < k1; ++kb) blk(S.lblk[kb]);
            }
        }
        hy[rr] = (double)h;
        sy[rr] = (double)s;
        zy[rr] = (double)z;
    }
}

template <int R, int NT, typename T>
__device__ __forceinline__ void store_rows(T *dst, const double (&v)[R], int n)
{
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
        const int i = threadIdx.x + rr * NT;
        if (i < n) dst[i] = (T)v[rr];
    }
}

template <int R, int NT>
__device__ __forceinline__ double dot_rows(const double (&a)[R], const double (&b)[R], int n)
{
    double s = 0.0;
#pragma unroll
    for (int rr = 0; rr < R; ++rr)
        if ((int)threadIdx.x + rr * NT < n) s += a[rr] * b[rr];
    return s;
}

// ------------------------------------------------------------------------
// inner CG: S_A s = e_j (a3), shared by both basis kernels
// ------------------------------------------------------------------------
// PREC 0: FP64 CG with true-residual restarts.  PREC 1, 2: FP32 CG passes
// with FP32 accumulation on the normalised FP64 residual, each judged and
// refined in FP64.  x holds the thread's rows of s_j on return.
template <int O, int R, int NT, int PREC>
__device__ void inner_cg(const DevSystem &S, const DevJob &J, const Col &g, int c, double *xa,
                         double *xb, double *red, float *redf, double (&x)[R], int &iters,
                         int &nres, int &status, int &start)
{
    constexpr int NWV = NT / 64;
    const int o = O ? O : S.o;
    const int tid = threadIdx.x;
    const int n = g.n;
    float *xaF = reinterpret_cast<float *>(xa);
    float *xbF = reinterpret_cast<float *>(xb);
    double dummy[R];
    bool converged = false;
    iters = nres = status = start = 0;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) x[rr] = 0.0;
    const int nout = kNbOut * o;
    if (J.x0) {
        // predicted coefficients on the orbitals of the kNbOut nearest atoms
        for (int i = tid; i < n; i += NT) xa[i] = 0.0;
        __syncthreads();
        for (int e = tid; e < nout; e += NT) {
            const int k = e / o, cc = e - k * o;
            const int la = S.out_loc[(int64_t)g.A * kNbOut + k];
            if (la >= 0) xa[la * o + cc] = (double)J.x0[(int64_t)c * nout + e];
        }
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int i = tid + rr * NT;
            if (i < n) x[rr] = xa[i];
        }
        start = 1;
        __syncthreads();
    }
    if (J.x0full) {
        // a start on the whole region (the kept s_j of an earlier solve)
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int i = tid + rr * NT;
            if (i < n) x[rr] = J.x0full[(int64_t)c * S.nmax + i];
        }
        start = 3;
    }
    if (PREC == 0) {
        double r[R], p[R], q[R];
        double rho2 = 1.0;
        if (start == 0) {
            // zero start: the residual is e_j itself
#pragma unroll
            for (int rr = 0; rr < R; ++rr) r[rr] = (tid + rr * NT) == g.jl ? 1.0 : 0.0;
        } else {
            // r = e_j - S x
            store_rows<R, NT, double>(xa, x, n);
            __syncthreads();
            spmv_rows<O, R, NT, double, double, false, true, false>(S, g, o, S.Hd, S.Sd, xa, xb, dummy, q, dummy);
#pragma unroll
            for (int rr = 0; rr < R; ++rr) r[rr] = ((tid + rr * NT) == g.jl ? 1.0 : 0.0) - q[rr];
            rho2 = block_sum<NWV>(dot_rows<R, NT>(r, r, n), red);
            ++nres;
        }
        if ((start == 1 || start == 3) && !(rho2 < 1.0)) {
            // the residual judge rejects the given start: zero start
            start += 1;
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                x[rr] = 0.0;
                r[rr] = (tid + rr * NT) == g.jl ? 1.0 : 0.0;
            }
            rho2 = 1.0;
        }
        for (int restart = 0; restart <= 3 && !converged && status == 0; ++restart) {
#pragma unroll
            for (int rr = 0; rr < R; ++rr) p[rr] = r[rr];
            for (int k = 0; k < n && sqrt(rho2) > J.cg_tol; ++k) {
                store_rows<R, NT, double>(xa, p, n);
                __syncthreads();
                spmv_rows<O, R, NT, double, double, false, true, false>(S, g, o, S.Hd, S.Sd, xa, xb, dummy, q, dummy);
                const double pq = block_sum<NWV>(dot_rows<R, NT>(p, q, n), red);
                if (!(pq > 0.0)) { status = -4; break; }
                const double alpha = rho2 / pq;
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    x[rr] += alpha * p[rr];
                    r[rr] -= alpha * q[rr];
                }
                const double rn = block_sum<NWV>(dot_rows<R, NT>(r, r, n), red);
                const double beta = rn / rho2;
#pragma unroll
                for (int rr = 0; rr < R; ++rr) p[rr] = r[rr] + beta * p[rr];
                rho2 = rn;
                ++iters;
            }
            if (status) break;
            // judge on the true residual
            store_rows<R, NT, double>(xa, x, n);
            __syncthreads();
            spmv_rows<O, R, NT, double, double, false, true, false>(S, g, o, S.Hd, S.Sd, xa, xb, dummy, q, dummy);
#pragma unroll
            for (int rr = 0; rr < R; ++rr) r[rr] = ((tid + rr * NT) == g.jl ? 1.0 : 0.0) - q[rr];
            rho2 = block_sum<NWV>(dot_rows<R, NT>(r, r, n), red);
            ++nres;
            if (sqrt(rho2) <= J.cg_tol) converged = true;
        }
    } else {
        double q[R], r64[R];
        for (int ref = 0; ref <= J.max_refine && status == 0; ++ref) {
            double rho2 = 1.0;
            if (ref == 0 && start == 0) {
                // zero start: the residual is e_j itself
#pragma unroll
                for (int rr = 0; rr < R; ++rr) r64[rr] = (tid + rr * NT) == g.jl ? 1.0 : 0.0;
            } else {
                store_rows<R, NT, double>(xa, x, n);
                __syncthreads();
                spmv_rows<O, R, NT, double, double, false, true, false>(S, g, o, S.Hd, S.Sd, xa, xb, dummy, q, dummy);
#pragma unroll
                for (int rr = 0; rr < R; ++rr) r64[rr] = ((tid + rr * NT) == g.jl ? 1.0 : 0.0) - q[rr];
                rho2 = block_sum<NWV>(dot_rows<R, NT>(r64, r64, n), red);
                ++nres;
            }
            if (ref == 0 && (start == 1 || start == 3) && !(rho2 < 1.0)) {
                start += 1;
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    x[rr] = 0.0;
                    r64[rr] = (tid + rr * NT) == g.jl ? 1.0 : 0.0;
                }
                rho2 = 1.0;
            }
            if (sqrt(rho2) <= J.cg_tol) { converged = true; break; }
            if (ref == J.max_refine) break;
            const double rho = sqrt(rho2);
            float rf[R], pf[R], df[R];
            double qd[R];
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                rf[rr] = (float)(r64[rr] / rho);
                pf[rr] = rf[rr];
                df[rr] = 0.0f;
            }
            float rrf = 0.0f;
#pragma unroll
            for (int rr = 0; rr < R; ++rr)
                if (tid + rr * NT < n) rrf += rf[rr] * rf[rr];
            rrf = block_sum<NWV>(rrf, redf);
            // relative target of the pass; no lower than what brings the
            // absolute residual to a tenth of cg_tol
            const float thr = (float)fmax(J.inner_tol, 0.1 * J.cg_tol / rho);
            for (int k = 0; k < n && sqrtf(rrf) > thr; ++k) {
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
                    if (tid + rr * NT < n) xaF[tid + rr * NT] = pf[rr];
                __syncthreads();
                spmv_rows<O, R, NT, float, float, false, true, false>(S, g, o, S.Hf, S.Sf, xaF, xbF, dummy, qd, dummy);
                float pq = 0.0f;
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
                    if (tid + rr * NT < n) pq += pf[rr] * (float)qd[rr];
                pq = block_sum<NWV>(pq, redf);
                if (!(pq > 0.0f)) { status = -4; break; }
                const float alpha = rrf / pq;
                float rn = 0.0f;
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    df[rr] += alpha * pf[rr];
                    rf[rr] -= alpha * (float)qd[rr];
                    if (tid + rr * NT < n) rn += rf[rr] * rf[rr];
                }
                rn = block_sum<NWV>(rn, redf);
                const float beta = rn / rrf;
#pragma unroll
                for (int rr = 0; rr < R; ++rr) pf[rr] = rf[rr] + beta * pf[rr];
                rrf = rn;
                ++iters;
            }
#pragma unroll
            for (int rr = 0; rr < R; ++rr) x[rr] += rho * (double)df[rr];
        }
    }
    if (status == 0 && !converged) status = -5;
    if (J.sj_store && status == 0) {
        // keep s_j for a later solve (MA_START_PREVIOUS)
        const int64_t jg = J.cols[c];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int i = tid + rr * NT;
            if (i < n) J.sj_store[jg * S.nmax + i] = x[rr];
        }
        if (tid == 0) J.sj_have[jg] = 1;
    }
    if (J.sj_near) {
        // s_j on the orbitals of the kNbOut nearest atoms (training targets)
        __syncthreads();
        store_rows<R, NT, double>(xa, x, n);
        __syncthreads();
        for (int e = tid; e < nout; e += NT) {
            const int k = e / o, cc = e - k * o;
            const int la = S.out_loc[(int64_t)g.A * kNbOut + k];
            J.sj_near[(int64_t)c * nout + e] = (status == 0 && la >= 0) ? (float)xa[la * o + cc] : 0.0f;
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void write_stats(const DevJob &J, int c, int L, int iters, int nres,
                                            int status, int start)
{
    int32_t *st = J.stats + (int64_t)c * kStats;
    st[0] = status == 0 ? L : 0;
    st[1] = iters;
    st[2] = nres;
    st[3] = status;
    st[4] = start;
    st[5] = st[6] = st[7] = 0;
    if (status != 0) atomicMin(J.fail, c);
}

// Persistent loop over the chunk's work queues: queue k serves order
// positions qbounds[k] .. qbounds[k+1]; a workgroup starts at queue
// blockIdx.x % nqueues (workgroups are dispatched to the XCDs round-robin)
// and moves on when a queue is exhausted.  Every queue is visited at most
// once, so every workgroup leaves the loop.
template <typename F>
__device__ __forceinline__ void drain_queues(const DevJob &J, int *s_idx, F &&body)
{
    int qi = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            int idx = -1;
            for (; qi < J.nqueues; ++qi) {
                const int k = (blockIdx.x + qi) % J.nqueues;
                const int pos = J.qbounds[k] + atomicAdd(J.queue + k, 1);
                if (pos < J.qbounds[k + 1]) { idx = pos; break; }
            }
            *s_idx = idx;
        }
        __syncthreads();
        const int idx = *s_idx;
        __syncthreads();
        if (idx < 0) break;
        body(J.order[idx], idx - J.c0);
    }
}

// The same loop over work items that are not single columns (the
// atom-group kernel: idx is a group position).
template <typename F>
__device__ __forceinline__ void drain_queues_raw(const DevJob &J, int *s_idx, F &&body)
{
    int qi = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            int idx = -1;
            for (; qi < J.nqueues; ++qi) {
                const int k = (blockIdx.x + qi) % J.nqueues;
                const int pos = J.qbounds[k] + atomicAdd(J.queue + k, 1);
                if (pos < J.qbounds[k + 1]) { idx = pos; break; }
            }
            *s_idx = idx;
        }
        __syncthreads();
        const int idx = *s_idx;
        __syncthreads();
        if (idx < 0) break;
        body(idx);
    }
}

// ------------------------------------------------------------------------
// large-region basis kernel: basis in the global workspace
// ------------------------------------------------------------------------
// Thread t owns local rows t, t + NTG, ...  The basis U, S U, H U and the
// block-2 chain T live in a per-workgroup slice of the global workspace
// (vector m at offset m * ld).  Each basis vector costs one fused dot sweep
// and one fused update sweep over the stored vectors: the S-orthogonalisation
// is classical Gram-Schmidt applied twice, with the second pass of each
// vector delayed into the step that projects the next candidate (the delayed
// reorthogonalisation of Bielich, Langou, Thomas, Swirydowicz, Yamazaki and
// Boman, Parallel Computing 112 (2022)).  Step s therefore
//   SpMV   S and H of the vector finalised in step s-1 (stored as S U, H U),
//          S of the pending vector (once projected), H of the next chain
//          source;
//   dots   a = (S U)^T pending, b = (S U)^T candidate, and for the chain
//          a_T = T^T pending chain vector, b_T = T^T (H of it);
//   update u = (pending - U a) / beta with beta^2 = pending^T S pending - |a|^2,
//          candidate - U b - u f becomes the next pending vector, where
//          f = u^T S candidate = (pending^T S candidate - a.b) / beta;
//          the chain likewise in the Euclidean inner product.
// The block-1 candidate is H applied to the pending vector rather than to
// the finished u: the two differ by H U a, which lies in the span already
// built (Krylov property of block 1) and is removed by the projections; the
// block-2 candidate is the pending chain vector, which differs from the
// finished t by a vector in the span of earlier chain vectors.  Breakdown
// (Eqs. 6-8 with the relative threshold tau) is judged on beta against the
// candidate's norm rebuilt from both passes' coefficients, as with two
// consecutive passes.

// Sum of 2 x 4 dot products per task: task g < nv covers V rows 4g..4g+3
// against x1, x2 (o1[m] = V[m].x1, o2[m] = V[m].x2), the remaining tasks W
// rows against y1, y2 (p1, p2).  Each wavefront takes whole tasks, so every
// basis vector is read once.
__device__ __forceinline__ void dot_sweep(const double *__restrict__ V, int LV, const double *x1,
                                          const double *x2, double *o1, double *o2,
                                          const double *__restrict__ W, int LW, const double *y1,
                                          const double *y2, double *p1, double *p2, int64_t ld,
                                          int n)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nv = (LV + 3) >> 2, nw = (LW + 3) >> 2;
    for (int task = w; task < nv + nw; task += NWG) {
        const bool first = task < nv;
        const int m0 = 4 * (first ? task : task - nv);
        const int L = first ? LV : LW;
        const int nm = min(4, L - m0);
        const double *B = first ? V : W;
        const double *X1 = first ? x1 : y1;
        const double *X2 = first ? x2 : y2;
        const double *v0 = B + m0 * ld;
        const double *v1 = B + (m0 + (nm > 1 ? 1 : 0)) * ld;
        const double *v2 = B + (m0 + (nm > 2 ? 2 : 0)) * ld;
        const double *v3 = B + (m0 + (nm > 3 ? 3 : 0)) * ld;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        double b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
        // four rows per lane and iteration: sixteen loads in flight
        for (int i0 = lane; i0 < n; i0 += 256) {
            double e[4][4], xv[4], zv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + 64 * r;
                const bool ok = i < n;
                const int ii = ok ? i : i0;
                e[r][0] = v0[ii];
                e[r][1] = v1[ii];
                e[r][2] = v2[ii];
                e[r][3] = v3[ii];
                xv[r] = ok ? X1[ii] : 0.0;
                zv[r] = ok ? X2[ii] : 0.0;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                a0 += e[r][0] * xv[r];
                a1 += e[r][1] * xv[r];
                a2 += e[r][2] * xv[r];
                a3 += e[r][3] * xv[r];
                b0 += e[r][0] * zv[r];
                b1 += e[r][1] * zv[r];
                b2 += e[r][2] * zv[r];
                b3 += e[r][3] * zv[r];
            }
        }
        double v[8] = {a0, a1, a2, a3, b0, b1, b2, b3};
        wave_transpose_reduce<8>(v);
        if (tr_writer<8>(lane)) {
            const int k = tr_index<8>(lane);
            const int m = m0 + (k & 3);
            double *dst = (k < 4) ? (first ? o1 : p1) : (first ? o2 : p2);
            if ((k & 3) < nm) dst[m] = v[0];
        }
    }
}

// s1[rr] = sum_m V[m][i] c1[m] and s2[rr] = sum_m V[m][i] c2[m] over m < cnt
// on the thread's rows i = tid + rr * NTG (rows at or past n read row 0; the
// caller discards them).  The loads of MB vectors are issued before their
// products, so MB R loads are in flight; the last batch is padded with
// copies of its first vector at coefficient zero, so every batch is one round
// trip (the sums are the same, term by term, as without the padding).
template <int R, int MB = 4>
__device__ __forceinline__ void comb2_rows(const double *__restrict__ V, int64_t ld, int cnt,
                                           const double *c1, const double *c2, int n,
                                           double (&s1)[R], double (&s2)[R])
{
    int off[R];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
        const int i = threadIdx.x + rr * NTG;
        off[rr] = i < n ? i : 0;
        s1[rr] = 0.0;
        s2[rr] = 0.0;
    }
    // MB vectors per batch: their loads are issued together (the last batch
    // is padded at coefficient zero, so every batch is one round trip)
    for (int m = 0; m < cnt; m += MB) {
        double v[MB][R];
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            const int mj = m + j < cnt ? m + j : m;
#pragma unroll
            for (int rr = 0; rr < R; ++rr) v[j][rr] = V[mj * ld + off[rr]];
        }
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            const bool ok = m + j < cnt;
            const int mj = ok ? m + j : m;
            const double a = ok ? c1[mj] : 0.0, b = ok ? c2[mj] : 0.0;
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                s1[rr] += v[j][rr] * a;
                s2[rr] += v[j][rr] * b;
            }
        }
    }
}

// SpMV of three staged vectors on the thread's own rows:
// ha = H xa, sa = S xa, sb = S xb, hd = H xd.
template <int O, int R, int NT, typename TM, typename TX>
__device__ __forceinline__ void spmv3_rows(const DevSystem &S, const Col &g, int o_rt,
                                           const TM *__restrict__ Hv, const TM *__restrict__ Sv,
                                           const TX *xa, const TX *xb, const TX *xd,
                                           double (&ha)[R], double (&sa)[R], double (&sb)[R],
                                           double (&hd)[R])
{
    const int o = O ? O : o_rt;
    constexpr int OB = O > 0 ? O : 1;   // the batched path below is taken for O > 0 only
    // blocks per batch: more value loads in flight per round trip, within
    // the registers of 2 waves per SIMD (9 x 9 FP32 blocks: 3 are 6 % faster
    // than 2 on the spd cell; 4 spill and are no faster)
    constexpr int NB = O > 4 ? (sizeof(TM) == 8 ? 2 : 3) : sizeof(TM) == 8 ? 3 : 4;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
        const int i = threadIdx.x + rr * NT;
        TX h1 = 0, s1 = 0, s2 = 0, h3 = 0;
        if (i < g.n) {
            const int a = i / o;
            const int ri = i - a * o;
            auto blk = [&](const int2 e) __attribute__((always_inline)) {
                const int64_t base = (int64_t)e.y * (o * o) + ri * o;
                const int xo = e.x * o;
                if constexpr (O > 0) {
#pragma unroll
                    for (int cc = 0; cc < O; ++cc) {
                        const TX hm = (TX)Hv[base + cc], sm = (TX)Sv[base + cc];
                        const TX va = xa[xo + cc];
                        h1 += hm * va;
                        s1 += sm * va;
                        s2 += sm * xb[xo + cc];
                        h3 += hm * xd[xo + cc];
                    }
                } else {
                    for (int cc = 0; cc < o; ++cc) {
                        const TX hm = (TX)Hv[base + cc], sm = (TX)Sv[base + cc];
                        const TX va = xa[xo + cc];
                        h1 += hm * va;
                        s1 += sm * va;
                        s2 += sm * xb[xo + cc];
                        h3 += hm * xd[xo + cc];
                    }
                }
            };
            if (g.lidx) {
                // batches of NB blocks: their value loads are issued before
                // any product (blocks past the row's end read its first
                // block and add nothing)
                const int k0 = g.srp[a], k1 = g.srp[a + 1];
                if constexpr (O == 0) {
                    for (int kb = k0; kb < k1; ++kb) blk(g.sblk[kb]);
                } else for (int kb = k0; kb < k1; kb += NB) {
                    int2 e[NB];
                    TM hm[NB][OB], sm[NB][OB];
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        e[j] = g.sblk[kb + j < k1 ? kb + j : k0];
                        const int64_t base = (int64_t)e[j].y * (o * o) + ri * o;
#pragma unroll
                        for (int cc = 0; cc < OB; ++cc) {
                            hm[j][cc] = Hv[base + cc];
                            sm[j][cc] = Sv[base + cc];
                        }
                    }
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        const bool ok = kb + j < k1;
                        const int xo = e[j].x * o;
#pragma unroll
                        for (int cc = 0; cc < OB; ++cc) {
                            const TX hv = ok ? (TX)hm[j][cc] : (TX)0;
                            const TX sv = ok ? (TX)sm[j][cc] : (TX)0;
                            const TX va = xa[xo + cc];
                            h1 += hv * va;
                            s1 += sv * va;
                            s2 += sv * xb[xo + cc];
                            h3 += hv * xd[xo + cc];
                        }
                    }
                }
            } else {
                const int64_t k0 = g.rp[a], k1 = g.rp[a + 1];
#pragma unroll 4
                for (int64_t kb = k0; kb < k1; ++kb) blk(S.lblk[kb]);
            }
        }
        ha[rr] = (double)h1;
        sa[rr] = (double)s1;
        sb[rr] = (double)s2;
        hd[rr] = (double)h3;
    }
}

struct SmemG {
    double *da, *dp, *dz, *dh;   // nmax each: SpMV input a, pending u, chain vector, H image
    void *fx;                    // PREC 1: the three SpMV inputs in FP32 (3 nmax floats)
    double *cf;                  // coefficients, 6 * (kMaxNu + 1)
    double *part;                // 4 * NWG wavefront partial sums
    double *red;                 // NWG
    float *redf;                 // NWG
    int *srp;                    // region block index (when staged): max_nat + 1 row pointers
    int2 *sblk;                  // and max_lnnz blocks
};

// candidate sources of a step
enum { kCandNone = 0, kCandBlock1 = 1, kCandChain = 2 };

template <int O, int R, int PREC>
__device__ void basis_global(const DevSystem &S, const DevJob &J, const SmemG &sm, int c, int s,
                             double *U, double *SU, double *K, double *T)
{
    using TM = typename std::conditional<PREC != 0, float, double>::type;
    using TX = typename std::conditional<PREC == 1, float, double>::type;
    const int o = O ? O : S.o;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t ld = S.nmax;
    const int nu = J.nu;
    Col g = make_col(S, J, c, o);
    if (J.lidx) stage_col_index<NTG>(S, g, sm.srp, sm.sblk);
    const int n = g.n;
    const TM *Hv = PREC ? (const TM *)S.Hf : (const TM *)S.Hd;
    const TM *Sv = PREC ? (const TM *)S.Sf : (const TM *)S.Sd;
    // SpMV inputs: a = finished vector, b = pending vector, d = H source
    TX *xa, *xb, *xz;
    if constexpr (PREC == 1) {
        xa = reinterpret_cast<TX *>(sm.fx);
        xb = xa + ld;
        xz = xb + ld;
    } else {
        xa = reinterpret_cast<TX *>(sm.da);
        xb = reinterpret_cast<TX *>(sm.dp);
        xz = reinterpret_cast<TX *>(sm.dz);
    }

    double x[R];
    int iters, nres, status, start;
    inner_cg<O, R, NTG, PREC>(S, J, g, c, sm.da, sm.dp, sm.red, sm.redf, x, iters, nres, status,
                              start);

    int L = 0;
    double *mid = J.mid + (int64_t)s * J.mid_stride;
    if (status == 0) {
        constexpr int CS = kMaxNu + 1;
        double *ca = sm.cf, *cbuf0 = ca + CS, *cbuf1 = cbuf0 + CS;
        double *cat = cbuf1 + CS, *ctb0 = cat + CS, *ctb1 = ctb0 + CS;
        // State between steps lives in LDS (rows owned by their thread):
        // xa the finished vector whose S and H images are not yet stored,
        // dp the pending vector (projected once, first-pass coefficients in
        // cp), dz the pending chain vector (projected once against T,
        // coefficients in ctp); with PREC 1, xb and xz hold FP32 copies of
        // dp and dz for the SpMV.
        bool has_fin = false, has_pend = J.p > 0;
        bool b1_live = true, chain_live = J.q > 0;
        int nb1 = J.p > 0 ? 1 : 0, k = 0, ping = 0;
        double cp_scale = 1.0, ctp_scale = 1.0;
        __syncthreads();   // the CG's last reads of da, dp are done
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int i = tid + rr * NTG;
            if (i < n) {
                const double e = (i == g.jl) ? 1.0 : 0.0;   // block 1 starts at e_j
                xa[i] = (TX)0.0;
                sm.dp[i] = e;
                sm.dz[i] = x[rr];                           // block 2 starts at s_j
                if constexpr (PREC == 1) {
                    xb[i] = (TX)e;
                    xz[i] = (TX)x[rr];
                }
            }
        }
        for (;;) {
            const int kind = (b1_live && nb1 < J.p) ? kCandBlock1
                             : chain_live ? kCandChain : kCandNone;
            if (!has_fin && !has_pend && kind == kCandNone) break;
            const bool need_z = kind == kCandChain && k + 1 < J.q;   // next raw chain vector
            const TX *xd = kind == kCandChain ? xz : xb;
            double *cb = ping ? cbuf1 : cbuf0, *cp = ping ? cbuf0 : cbuf1;
            double *ctb = ping ? ctb1 : ctb0, *ctp = ping ? ctb0 : ctb1;

            // ---- SpMV ----
            __syncthreads();   // staged vectors visible
            double hf[R], sf[R], sp[R], hz[R];
            spmv3_rows<O, R, NTG, TM, TX>(S, g, o, Hv, Sv, xa, xb, xd, hf, sf, sp, hz);
            if (has_fin) {
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    const int i = tid + rr * NTG;
                    if (i < n) {
                        SU[(L - 1) * ld + i] = sf[rr];
                        K[(L - 1) * ld + i] = hf[rr];
                    }
                }
            }
            if (kind == kCandNone && !has_pend) break;   // tail: images of the last vector stored
            // row-local parts of pending^T S pending, pending^T S candidate,
            // chain^T chain, chain^T (H chain)
            double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int i = tid + rr * NTG;
                if (i < n) {
                    const double up = sm.dp[i], zt = sm.dz[i];
                    const double cand = kind == kCandChain ? zt : hz[rr];
                    sm.dh[i] = hz[rr];
                    q0 += up * sp[rr];
                    q1 += sp[rr] * cand;
                    q2 += zt * zt;
                    q3 += zt * hz[rr];
                }
            }
            {
                double v[4] = {q0, q1, q2, q3};
                wave_transpose_reduce<4>(v);
                if (tr_writer<4>(lane)) sm.part[wv * 4 + tr_index<4>(lane)] = v[0];
            }
            __syncthreads();   // LDS inputs, partials and the S U, H U rows visible

            // ---- dots ----
            const int Lb = kind != kCandNone ? L : 0;   // candidate dots
            const int La = has_pend ? L : 0;            // reorthogonalisation dots
            const int kt = kind == kCandChain ? k : 0;
            dot_sweep(SU, max(La, Lb), sm.dp, kind == kCandChain ? sm.dz : sm.dh, ca, cb, T, kt,
                      sm.dz, sm.dh, cat, ctb, ld, n);
            __syncthreads();

            // ---- decisions (every thread, same values) ----
            double nu_p = 0.0, e_p = 0.0, nu_t = 0.0, e_t = 0.0;
#pragma unroll
            for (int w = 0; w < NWG; ++w) {
                nu_p += sm.part[w * 4 + 0];
                e_p += sm.part[w * 4 + 1];
                nu_t += sm.part[w * 4 + 2];
                e_t += sm.part[w * 4 + 3];
            }
            // Candidates are rescaled as they are projected (block 1: H u =
            // H pending / beta; chain: H t = H chain / eta), so the stored
            // first-pass coefficients refer to the unscaled vectors and are
            // multiplied by the scale when the rebuilt norm is formed.
            bool acc_u = false;
            double beta = 1.0, f = 0.0;
            if (has_pend) {
                double asq = 0.0, tot = 0.0, ab = 0.0;
                for (int m = 0; m < L; ++m) {
                    const double cm = cp_scale * cp[m] + ca[m];
                    asq += ca[m] * ca[m];
                    tot += cm * cm;
                    if (kind != kCandNone) ab += ca[m] * cb[m];
                }
                const double bb = nu_p - asq, b0 = bb + tot;
                acc_u = bb > 0.0 && b0 > 0.0 && !(sqrt(bb) <= J.tau * sqrt(b0));
                if (acc_u) {
                    beta = sqrt(bb);
                    f = (e_p - ab) / beta;
                }
            }
            bool acc_t = false;
            double eta = 1.0, ft = 0.0;
            if (kind == kCandChain) {
                double asq = 0.0, tot = 0.0, ab = 0.0;
                for (int m = 0; m < k; ++m) {
                    const double cm = ctp_scale * ctp[m] + cat[m];
                    asq += cat[m] * cat[m];
                    tot += cm * cm;
                    ab += cat[m] * ctb[m];
                }
                const double ee = nu_t - asq, e0 = ee + tot;
                acc_t = ee > 0.0 && sqrt(ee) > J.tau * sqrt(e0);
                if (acc_t) {
                    eta = sqrt(ee);
                    ft = (e_t - ab) / eta;
                }
            }
            // a block-1 candidate is H of the pending vector: void if that broke down
            const bool new_pend = (kind == kCandBlock1 && acc_u) || (kind == kCandChain && acc_t);
            const bool new_chain = need_z && acc_t;
            const double inv_b = 1.0 / beta, inv_e = 1.0 / eta;
            const double sc = kind == kCandBlock1 ? inv_b : 1.0;

            // ---- update sweep: finish u and t, project the candidates once ----
            double sa[R], sb[R], ta[R], tb[R];
            comb2_rows<R>(U, ld, (acc_u || new_pend) ? L : 0, ca, cb, n, sa, sb);
            comb2_rows<R>(T, ld, acc_t ? k : 0, cat, ctb, n, ta, tb);
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int i = tid + rr * NTG;
                if (i < n) {
                    const double up = sm.dp[i], zt = sm.dz[i], hv = sm.dh[i];
                    const double u = (up - sa[rr]) * inv_b;
                    const double cand = kind == kCandChain ? zt : hv;
                    const double nl = (cand - sb[rr] - (acc_u ? f * u : 0.0)) * sc;
                    const double t = (zt - ta[rr]) * inv_e;
                    const double nz = (hv - tb[rr] - ft * t) * inv_e;
                    if (acc_t) T[k * ld + i] = t;
                    if (acc_u) {
                        U[L * ld + i] = u;
                        xa[i] = (TX)u;
                    }
                    const double pn = new_pend ? nl : 0.0;
                    sm.dp[i] = pn;
                    if constexpr (PREC == 1) xb[i] = (TX)pn;
                    if (new_chain) {
                        sm.dz[i] = nz;
                        if constexpr (PREC == 1) xz[i] = (TX)nz;
                    }
                }
            }
            if (tid == 0) {
                if (acc_u) cb[L] = f;    // coefficient of the new pending vector on u_L
                if (acc_t) ctb[k] = ft;
            }
            if (kind == kCandBlock1) {
                if (acc_u) ++nb1;
                else b1_live = false;
            }
            if (kind == kCandChain) {
                if (acc_t) {
                    ++k;
                    chain_live = k < J.q;
                } else {
                    chain_live = false;
                }
            }
            if (acc_u) ++L;
            cp_scale = sc;
            ctp_scale = inv_e;
            has_fin = acc_u;
            has_pend = new_pend;
            ping ^= 1;
        }
        __syncthreads();   // basis writes visible to the whole workgroup

        // ---------------- Galerkin pair X = U^T K, S~ = U^T SU ----------------
        // Dense L x L products on the FP64 matrix cores: 16 x 16 output tiles,
        // v_mfma_f64_16x16x4f64 over the region rows, one tile per wavefront
        // at a time.  Lane l feeds A[l%16][l/16] = u_m[i] and
        // B[l/16][l%16] = k_n[i] (resp. (S u_n)[i]) and receives
        // D[4*j + l/16][l%16], j = 0..3.  Both triangles are written; the
        // eigensolver symmetrises.
        double *Xh = mid, *Xs = mid + (int64_t)nu * nu;
        {
            const int nt = (L + 15) >> 4;
            for (int tile = wv; tile < nt * nt; tile += NWG) {
                const int mt = tile / nt, ntc = tile - mt * nt;
                const int m = mt * 16 + (lane & 15), nn = ntc * 16 + (lane & 15);
                const int kk = lane >> 4;
                const bool mok = m < L, nok = nn < L;
                const double *um = U + (int64_t)(mok ? m : 0) * ld;
                const double *kn = K + (int64_t)(nok ? nn : 0) * ld;
                const double *sn = SU + (int64_t)(nok ? nn : 0) * ld;
                dbl4 ah = {0.0, 0.0, 0.0, 0.0}, as = {0.0, 0.0, 0.0, 0.0};
                // eight k-steps per batch: their 24 loads are issued together
                for (int i0 = 0; i0 < n; i0 += 32) {
                    double av[8], hv8[8], sv8[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int i = i0 + 4 * u + kk;
                        const bool iok = i < n;
                        av[u] = (mok && iok) ? um[i] : 0.0;
                        hv8[u] = (nok && iok) ? kn[i] : 0.0;
                        sv8[u] = (nok && iok) ? sn[i] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        ah = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], hv8[u], ah, 0, 0, 0);
                        as = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], sv8[u], as, 0, 0, 0);
                    }
                }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int mr = mt * 16 + 4 * jj + kk, nc = ntc * 16 + (lane & 15);
                    if (mr < L && nc < L) {
                        Xh[mr * nu + nc] = ah[jj];
                        Xs[mr * nu + nc] = as[jj];
                    }
                }
            }
        }
        // rows of U the outputs need: u at row j, S u at row j, u at the pattern rows
        double *Up = mid + 2 * (int64_t)nu * nu;
        const int64_t kb0 = S.blk_ptr[g.A];
        const int npat = (int)(S.blk_ptr[g.A + 1] - kb0) * o;
        for (int e = tid; e < (npat + 2) * L; e += NTG) {
            const int row = e / L, m = e - row * L;
            double v;
            if (row == 0) v = U[m * ld + g.jl];
            else if (row == 1) v = SU[m * ld + g.jl];
            else {
                const int tt = row - 2;
                v = U[m * ld + S.blk_loc[kb0 + tt / o] * o + (tt % o)];
            }
            Up[row * nu + m] = v;
        }
    }
    if (tid == 0) write_stats(J, c, L, iters, nres, status, start);
    __syncthreads();
}

// LDS of the workspace kernel, in doubles: four vectors, the FP32 SpMV inputs
// of PREC 1 (1.5 vectors) and the coefficients
__host__ __device__ constexpr int64_t global_smem_doubles(int64_t nmax)
{
    return 4 * nmax + (3 * nmax + 1) / 2 + 6 * (kMaxNu + 1) + 4 * NWG;
}

// waves per SIMD the register allocation aims at: 2 (with 3 the basis kernel
// alone is faster, but it leaves no room for the eigensolver of the previous
// chunk, and the pipelined solve is slower)
constexpr int kGlobalWaves = 2;

template <int O, int R, int PREC>
__global__ void __launch_bounds__(NTG, kGlobalWaves) k_basis_g(DevSystem S, DevJob J)
{
    extern __shared__ double smem[];
    __shared__ double red[NWG];
    __shared__ float redf[NWG];
    __shared__ int s_idx;
    const int64_t nm = S.nmax;
    SmemG sm;
    sm.da = smem;
    sm.dp = smem + nm;
    sm.dz = smem + 2 * nm;
    sm.dh = smem + 3 * nm;
    sm.fx = smem + 4 * nm;
    sm.cf = smem + 4 * nm + (3 * nm + 1) / 2;
    sm.part = sm.cf + 6 * (kMaxNu + 1);
    sm.srp = reinterpret_cast<int *>(sm.part + 4 * NWG);
    sm.sblk = reinterpret_cast<int2 *>(sm.srp + ((S.max_nat + 2) & ~1));
    sm.red = red;
    sm.redf = redf;
    double *U = J.ws + (int64_t)blockIdx.x * J.ws_stride;
    double *SU = U + J.nu * nm;
    double *K = SU + J.nu * nm;
    double *T = K + J.nu * nm;
    drain_queues(J, &s_idx, [&](int c, int s) __attribute__((always_inline)) {
        basis_global<O, R, PREC>(S, J, sm, c, s, U, SU, K, T);
    });
}

// ------------------------------------------------------------------------
// atom-group basis kernel: the columns of one atom in lockstep
// ------------------------------------------------------------------------
// The columns j = (A, r) of atom A share its region and region operator.
// One workgroup runs their CGs, Gram-Schmidt recurrences and Galerkin
// projections together: every SpMV is an SpMM that reads each operator value
// once for all of them, and every workgroup reduction carries one value per
// column.  Each column keeps its own basis (U, S U, H U, chain) in the
// workspace; CG convergence and breakdowns are per column (masks).  Thread t
// owns local rows t, t + NT, ...; the B vectors an SpMM reads are staged in
// LDS, vector k at offset k * ldx.

// pad B values to a power of two for the transposed reduction
template <int B>
__host__ __device__ constexpr int pow2_at_least() { return B <= 1 ? 1 : B <= 2 ? 2 : B <= 4 ? 4 : B <= 8 ? 8 : 16; }

// out[k] = sum over the workgroup of v[k], k < B (LDS `out`, B entries).
template <int NWV, int B, typename F>
__device__ __forceinline__ void group_sum(F &&gen, double *scratch, double *out)
{
    constexpr int NV = pow2_at_least<B>();
    block_reduce<NWV, NV, 1>([&](int, double (&v)[NV]) __attribute__((always_inline)) {
        double t[B];
        gen(t);
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = k < B ? t[k] : 0.0;
    }, scratch, out);
}

// Fused SpMM on the thread's rows: hy[k] = H xa_k, sy[k] = S xa_k, zy[k] = H xb_k.
template <int O, int R, int NT, int B, typename TM, typename TX, bool DO_H, bool DO_S, bool DO_Z>
__device__ __forceinline__ void spmm_rows(const DevSystem &S, const Col &g, const TM *__restrict__ Hv,
                                          const TM *__restrict__ Sv, const TX *xa, const TX *xb,
                                          int ldx, double (&hy)[R][B], double (&sy)[R][B],
                                          double (&zy)[R][B])
{
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
        const int i = threadIdx.x + rr * NT;
        TX h[B], s[B], z[B];
#pragma unroll
        for (int k = 0; k < B; ++k) h[k] = s[k] = z[k] = 0;
        if (i < g.n) {
            const int a = i / O;
            const int ri = i - a * O;
            const int64_t k0 = g.rp[a], k1 = g.rp[a + 1];
#pragma unroll 4
            for (int64_t kb = k0; kb < k1; ++kb) {
                const int2 e = S.lblk[kb];
                const int64_t base = (int64_t)e.y * (O * O) + ri * O;
                const int xo = e.x * O;
#pragma unroll
                for (int cc = 0; cc < O; ++cc) {
                    const TX hvv = DO_H || DO_Z ? (TX)Hv[base + cc] : (TX)0;
                    const TX svv = DO_S ? (TX)Sv[base + cc] : (TX)0;
#pragma unroll
                    for (int k = 0; k < B; ++k) {
                        if (DO_H) h[k] += hvv * xa[k * ldx + xo + cc];
                        if (DO_S) s[k] += svv * xa[k * ldx + xo + cc];
                        if (DO_Z) z[k] += hvv * xb[k * ldx + xo + cc];
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            hy[rr][k] = (double)h[k];
            sy[rr][k] = (double)s[k];
            zy[rr][k] = (double)z[k];
        }
    }
}

// out[k * kMaxNu + m] = V_k[m] . x_k for k < nb, m < cnt[k] (x_k in LDS at
// k * ldx).  The dot products of all columns are spread over the wavefronts,
// four consecutive ones at a time.
template <int NWV, int B>
__device__ __forceinline__ void multidot_group(double *const (&V)[B], int64_t ld, const int (&cnt)[B],
                                               int nb, const double *x, int ldx, int n, double *out)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int total = 0;
#pragma unroll
    for (int k = 0; k < B; ++k) total += k < nb ? cnt[k] : 0;
    for (int t0 = 4 * w; t0 < total; t0 += 4 * NWV) {
        const double *vp[4];
        const double *xp[4];
        int dst[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int t = t0 + u < total ? t0 + u : t0;
            int kk = 0;
#pragma unroll
            for (int k = 0; k < B; ++k)
                if (k < nb && t >= cnt[k] && kk == k) {
                    t -= cnt[k];
                    kk = k + 1;
                }
            vp[u] = V[0];
            xp[u] = x;
#pragma unroll
            for (int k = 0; k < B; ++k)
                if (k == kk) {
                    vp[u] = V[k] + (int64_t)t * ld;
                    xp[u] = x + k * ldx;
                }
            dst[u] = t0 + u < total ? kk * kMaxNu + t : -1;
        }
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        for (int i = lane; i < n; i += 64) {
            a0 += vp[0][i] * xp[0][i];
            a1 += vp[1][i] * xp[1][i];
            a2 += vp[2][i] * xp[2][i];
            a3 += vp[3][i] * xp[3][i];
        }
        a0 = wave_sum(a0);
        a1 = wave_sum(a1);
        a2 = wave_sum(a2);
        a3 = wave_sum(a3);
        if (lane == 0) {
            if (dst[0] >= 0) out[dst[0]] = a0;
            if (dst[1] >= 0) out[dst[1]] = a1;
            if (dst[2] >= 0) out[dst[2]] = a2;
            if (dst[3] >= 0) out[dst[3]] = a3;
        }
    }
}

struct SmemM {
    double *xa, *xb;     // B * ldx doubles each: staged vectors
    double *cf;          // 2 * B * kMaxNu: Gram-Schmidt coefficients per column
    double *gs;          // group sums (up to 16 values)
    double *scratch;     // transposed-reduction scratch
    int ldx;
};

template <int O, int B, int NT, int R, int PREC>
__device__ void basis_group(const DevSystem &S, const DevJob &J, const SmemM &sm, int gpos,
                            double *ws)
{
    constexpr int NWV = NT / 64;
    using TM = typename std::conditional<PREC != 0, float, double>::type;
    using TX = typename std::conditional<PREC == 1, float, double>::type;
    const int tid = threadIdx.x;
    const int nu = J.nu;
    const int64_t ld = S.nmax;
    const int ldx = sm.ldx;
    const int p0 = J.gstart[gpos];
    const int nb = J.gstart[gpos + 1] - p0;
    // the group's columns: output rows, slots and orbitals
    int cc_[B], slot[B], orb[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
        const int pos = p0 + (k < nb ? k : 0);
        cc_[k] = J.order[pos];
        slot[k] = pos - J.c0;
        orb[k] = J.cols[cc_[k]] % O;
    }
    const int A = J.cols[cc_[0]] / O;
    Col g;
    {
        const int rid = S.reg_id[A];
        g.A = A;
        g.r = 0;
        g.n_at = S.reg_len[rid];
        g.n = g.n_at * O;
        g.rp = S.lrp + S.lrp_off[rid];
        g.jl = S.jloc[A] * O;   // local row of orbital 0 of atom A
    }
    const int n = g.n;
    int jl[B];
#pragma unroll
    for (int k = 0; k < B; ++k) jl[k] = g.jl + orb[k];
    auto valid = [&](int k) __attribute__((always_inline)) { return k < nb; };
    auto own = [&](int rr) __attribute__((always_inline)) { return tid + rr * NT < n; };
    auto unit = [&](int rr, int k) __attribute__((always_inline)) {
        return (tid + rr * NT) == jl[k] ? 1.0 : 0.0;
    };
    double *gs = sm.gs;
    double dmy[R][B];

    // ---------------- inner CGs: S_A s_k = e_jk, in lockstep ----------------
    double x[R][B];
    int iters[B], nres[B], status[B], start[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
        iters[k] = nres[k] = start[k] = 0;
        status[k] = valid(k) ? 0 : 1;   // 1: not a column of this group
#pragma unroll
        for (int rr = 0; rr < R; ++rr) x[rr][k] = 0.0;
    }
    const int nout = kNbOut * O;
    if (J.x0) {
        for (int e = tid; e < B * ldx; e += NT) sm.xa[e] = 0.0;
        __syncthreads();
        for (int e = tid; e < nb * nout; e += NT) {
            const int k = e / nout, f = e - k * nout;
            const int kn = f / O, c2 = f - kn * O;
            const int la = S.out_loc[(int64_t)A * kNbOut + kn];
            int ck = cc_[0];
#pragma unroll
            for (int kk = 0; kk < B; ++kk)
                if (kk == k) ck = cc_[kk];
            if (la >= 0) sm.xa[k * ldx + la * O + c2] = (double)J.x0[(int64_t)ck * nout + f];
        }
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int k = 0; k < B; ++k)
                if (own(rr) && valid(k)) x[rr][k] = sm.xa[k * ldx + tid + rr * NT];
#pragma unroll
        for (int k = 0; k < B; ++k)
            if (valid(k)) start[k] = 1;
        __syncthreads();
    }
    // stage x (FP64), S x for every column
    auto stage64 = [&](const double (&v)[R][B], double *dst) __attribute__((always_inline)) {
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int k = 0; k < B; ++k)
                if (own(rr)) dst[k * ldx + tid + rr * NT] = v[rr][k];
    };
    double q[R][B], rv[R][B];
    auto true_residual = [&]() __attribute__((always_inline)) {
        stage64(x, sm.xa);
        __syncthreads();
        spmm_rows<O, R, NT, B, double, double, false, true, false>(S, g, S.Hd, S.Sd, sm.xa, sm.xb, ldx, dmy, q, dmy);
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int k = 0; k < B; ++k) rv[rr][k] = unit(rr, k) - q[rr][k];
        group_sum<NWV, B>([&](double (&t)[B]) __attribute__((always_inline)) {
#pragma unroll
            for (int k = 0; k < B; ++k) {
                double a = 0.0;
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
                    if (own(rr)) a += rv[rr][k] * rv[rr][k];
                t[k] = a;
            }
        }, sm.scratch, gs);
    };
    double rho2[B];
    bool conv[B];
#pragma unroll
    for (int k = 0; k < B; ++k) conv[k] = false;
    true_residual();
#pragma unroll
    for (int k = 0; k < B; ++k) {
        rho2[k] = gs[k];
        if (valid(k)) ++nres[k];
        if (valid(k) && start[k] == 1 && !(rho2[k] < 1.0)) {
            // the residual judge rejects the predicted start: zero start
            start[k] = 2;
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                x[rr][k] = 0.0;
                rv[rr][k] = unit(rr, k);
            }
            rho2[k] = 1.0;
        }
    }
    if (PREC == 0) {
        double pv[R][B];
        for (int restart = 0; restart <= 3; ++restart) {
            bool any = false;
#pragma unroll
            for (int k = 0; k < B; ++k) any |= status[k] == 0 && !conv[k];
            if (!any) break;
#pragma unroll
            for (int rr = 0; rr < R; ++rr)
#pragma unroll
                for (int k = 0; k < B; ++k) pv[rr][k] = rv[rr][k];
            int it[B];
#pragma unroll
            for (int k = 0; k < B; ++k) it[k] = 0;
            for (;;) {
                bool act[B];
                bool anyact = false;
#pragma unroll
                for (int k = 0; k < B; ++k) {
                    act[k] = status[k] == 0 && !conv[k] && it[k] < n && sqrt(rho2[k]) > J.cg_tol;
                    anyact |= act[k];
                }
                if (!anyact) break;
                stage64(pv, sm.xa);
                __syncthreads();
                spmm_rows<O, R, NT, B, double, double, false, true, false>(S, g, S.Hd, S.Sd, sm.xa, sm.xb, ldx, dmy, q, dmy);
                group_sum<NWV, B>([&](double (&t)[B]) __attribute__((always_inline)) {
#pragma unroll
                    for (int k = 0; k < B; ++k) {
                        double a = 0.0;
#pragma unroll
                        for (int rr = 0; rr < R; ++rr)
                            if (own(rr)) a += pv[rr][k] * q[rr][k];
                        t[k] = a;
                    }
                }, sm.scratch, gs);
                double alpha[B];
#pragma unroll
                for (int k = 0; k < B; ++k) {
                    const double pq = gs[k];
                    alpha[k] = 0.0;
                    if (act[k]) {
                        if (!(pq > 0.0)) {
                            status[k] = -4;
                            act[k] = false;
                        } else {
                            alpha[k] = rho2[k] / pq;
                        }
                    }
#pragma unroll
                    for (int rr = 0; rr < R; ++rr)
                        if (act[k]) {
                            x[rr][k] += alpha[k] * pv[rr][k];
                            rv[rr][k] -= alpha[k] * q[rr][k];
                        }
                }
                group_sum<NWV, B>([&](double (&t)[B]) __attribute__((always_inline)) {
#pragma unroll
                    for (int k = 0; k < B; ++k) {
                        double a = 0.0;
#pragma unroll
                        for (int rr = 0; rr < R; ++rr)
                            if (own(rr)) a += rv[rr][k] * rv[rr][k];
                        t[k] = a;
                    }
                }, sm.scratch, gs);
#pragma unroll
                for (int k = 0; k < B; ++k)
                    if (act[k]) {
                        const double rn = gs[k];
                        const double beta = rn / rho2[k];
#pragma unroll
                        for (int rr = 0; rr < R; ++rr) pv[rr][k] = rv[rr][k] + beta * pv[rr][k];
                        rho2[k] = rn;
                        ++iters[k];
                        ++it[k];
                    }
            }
            // judge on the true residual
            true_residual();
#pragma unroll
            for (int k = 0; k < B; ++k)
                if (status[k] == 0 && !conv[k]) {
                    rho2[k] = gs[k];
                    ++nres[k];
                    if (sqrt(rho2[k]) <= J.cg_tol) conv[k] = true;
                }
        }
    } else {
        // FP32 CG passes on the normalised FP64 residual, refined in FP64
        TX *xaX = reinterpret_cast<TX *>(sm.xa);
        float *xaF = reinterpret_cast<float *>(sm.xa);
        for (int ref = 0; ref <= J.max_refine; ++ref) {
            if (ref > 0) {
                true_residual();
#pragma unroll
                for (int k = 0; k < B; ++k)
                    if (status[k] == 0 && !conv[k]) {
                        rho2[k] = gs[k];
                        ++nres[k];
                    }
            }
            bool any = false;
#pragma unroll
            for (int k = 0; k < B; ++k) {
                if (status[k] == 0 && !conv[k] && sqrt(rho2[k]) <= J.cg_tol) conv[k] = true;
                any |= status[k] == 0 && !conv[k];
            }
            if (!any || ref == J.max_refine) break;
            double rho[B];
            float rf[R][B], pf[R][B], df[R][B];
            float rrf[B];
#pragma unroll
            for (int k = 0; k < B; ++k) {
                rho[k] = sqrt(rho2[k]);
                rrf[k] = 0.0f;
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    const bool on = status[k] == 0 && !conv[k];
                    rf[rr][k] = on ? (float)(rv[rr][k] / rho[k]) : 0.0f;
                    pf[rr][k] = rf[rr][k];
                    df[rr][k] = 0.0f;
                }
            }
            group_sum<NWV, B>([&](double (&t)[B]) __attribute__((always_inline)) {
#pragma unroll
                for (int k = 0; k < B; ++k) {
                    float a = 0.0f;
#pragma unroll
                    for (int rr = 0; rr < R; ++rr)
                        if (own(rr)) a += rf[rr][k] * rf[rr][k];
                    t[k] = (double)a;
                }
            }, sm.scratch, gs);
#pragma unroll
            for (int k = 0; k < B; ++k) rrf[k] = (float)gs[k];
            float thr[B];
#pragma unroll
            for (int k = 0; k < B; ++k) thr[k] = (float)fmax(J.inner_tol, 0.1 * J.cg_tol / rho[k]);
            int it[B];
#pragma unroll
            for (int k = 0; k < B; ++k) it[k] = 0;
            for (;;) {
                bool act[B];
                bool anyact = false;
#pragma unroll
                for (int k = 0; k < B; ++k) {
                    act[k] = status[k] == 0 && !conv[k] && it[k] < n && sqrtf(rrf[k]) > thr[k];
                    anyact |= act[k];
                }
                if (!anyact) break;
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
#pragma unroll
                    for (int k = 0; k < B; ++k)
                        if (own(rr)) xaF[k * ldx + tid + rr * NT] = pf[rr][k];
                __syncthreads();
                float qf[R][B];
                {
                    double qd[R][B];
                    spmm_rows<O, R, NT, B, float, float, false, true, false>(S, g, S.Hf, S.Sf, xaF, xaF, ldx, dmy, qd, dmy);
#pragma unroll
                    for (int rr = 0; rr < R; ++rr)
#pragma unroll
                        for (int k = 0; k < B; ++k) qf[rr][k] = (float)qd[rr][k];
                }
                group_sum<NWV, B>([&](double (&t)[B]) __attribute__((always_inline)) {
#pragma unroll
                    for (int k = 0; k < B; ++k) {
                        float a = 0.0f;
#pragma unroll
                        for (int rr = 0; rr < R; ++rr)
                            if (own(rr)) a += pf[rr][k] * qf[rr][k];
                        t[k] = (double)a;
                    }
                }, sm.scratch, gs);
#pragma unroll
                for (int k = 0; k < B; ++k) {
                    const float pq = (float)gs[k];
                    float alpha = 0.0f;
                    if (act[k]) {
                        if (!(pq > 0.0f)) {
                            status[k] = -4;
                            act[k] = false;
                        } else {
                            alpha = rrf[k] / pq;
                        }
                    }
#pragma unroll
                    for (int rr = 0; rr < R; ++rr)
                        if (act[k]) {
                            df[rr][k] += alpha * pf[rr][k];
                            rf[rr][k] -= alpha * qf[rr][k];
                        }
                }
                group_sum<NWV, B>([&](double (&t)[B]) __attribute__((always_inline)) {
#pragma unroll
                    for (int k = 0; k < B; ++k) {
                        float a = 0.0f;
#pragma unroll
                        for (int rr = 0; rr < R; ++rr)
                            if (own(rr)) a += rf[rr][k] * rf[rr][k];
                        t[k] = (double)a;
                    }
                }, sm.scratch, gs);
#pragma unroll
                for (int k = 0; k < B; ++k)
                    if (act[k]) {
                        const float rn = (float)gs[k];
                        const float beta = rn / rrf[k];
#pragma unroll
                        for (int rr = 0; rr < R; ++rr) pf[rr][k] = rf[rr][k] + beta * pf[rr][k];
                        rrf[k] = rn;
                        ++iters[k];
                        ++it[k];
                    }
            }
#pragma unroll
            for (int k = 0; k < B; ++k)
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
                    if (status[k] == 0 && !conv[k]) x[rr][k] += rho[k] * (double)df[rr][k];
        }
        (void)xaX;
    }
#pragma unroll
    for (int k = 0; k < B; ++k)
        if (status[k] == 0 && !conv[k]) status[k] = -5;
    if (J.sj_near) {
        __syncthreads();
        stage64(x, sm.xa);
        __syncthreads();
        for (int e = tid; e < nb * nout; e += NT) {
            const int k = e / nout, f = e - k * nout;
            const int kn = f / O, c2 = f - kn * O;
            const int la = S.out_loc[(int64_t)A * kNbOut + kn];
            int ck = cc_[0], stk = 0;
#pragma unroll
            for (int kk = 0; kk < B; ++kk)
                if (kk == k) {
                    ck = cc_[kk];
                    stk = status[kk];
                }
            J.sj_near[(int64_t)ck * nout + f] = (stk == 0 && la >= 0) ? (float)sm.xa[k * ldx + la * O + c2] : 0.0f;
        }
        __syncthreads();
    }

    // ---------------- bases of K_p(H;e_j) + K_q(H;s_j), in lockstep ----------------
    const int64_t cstride = (int64_t)(3 * nu + J.q) * ld;
    double *U[B], *SU[B], *K[B], *T[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
        U[k] = ws + k * cstride;
        SU[k] = U[k] + nu * ld;
        K[k] = SU[k] + nu * ld;
        T[k] = K[k] + nu * ld;
    }
    // first chain vector t_1 = s_j / |s_j| (kept in the workspace; s_j dies here)
    if (J.q > 0) {
        group_sum<NWV, B>([&](double (&tt)[B]) __attribute__((always_inline)) {
#pragma unroll
            for (int k = 0; k < B; ++k) {
                double a = 0.0;
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
                    if (own(rr)) a += x[rr][k] * x[rr][k];
                tt[k] = a;
            }
        }, sm.scratch, gs);
#pragma unroll
        for (int k = 0; k < B; ++k) {
            if (status[k] != 0) continue;
            const double ns = sqrt(gs[k]);
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int i = tid + rr * NT;
                if (i < n) T[k][i] = x[rr][k] / ns;
            }
        }
    }
    int L[B];
#pragma unroll
    for (int k = 0; k < B; ++k) L[k] = 0;
    double l[R][B], zv[R][B];
    double *c1 = sm.cf, *c2 = sm.cf + B * kMaxNu;
    TX *xaX = reinterpret_cast<TX *>(sm.xa);
    TX *xbX = reinterpret_cast<TX *>(sm.xb);
    const TM *Hv = PREC ? (const TM *)S.Hf : (const TM *)S.Hd;
    const TM *Sv = PREC ? (const TM *)S.Sf : (const TM *)S.Sd;

    // One candidate per active column (Eqs. 6-8): two classical Gram-Schmidt
    // passes with coefficients u_m^T S l, S-normalisation, breakdown test,
    // acceptance u = l/beta, S u, H u.  With `chain`, also zv = H t.  Returns
    // the mask of accepted columns.
    auto append = [&](const bool (&act)[B], bool chain, int kk) __attribute__((always_inline)) -> unsigned {
        int cnt[B];
#pragma unroll
        for (int k = 0; k < B; ++k) cnt[k] = act[k] ? L[k] : 0;
        for (int pass = 0; pass < 2; ++pass) {
            double *cc = pass ? c2 : c1;
            stage64(l, sm.xa);
            __syncthreads();
            multidot_group<NWV, B>(SU, ld, cnt, nb, sm.xa, ldx, n, cc);
            __syncthreads();
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int i = tid + rr * NT;
                if (i < n) {
#pragma unroll
                    for (int k = 0; k < B; ++k) {
                        double acc = 0.0;
                        for (int m = 0; m < cnt[k]; ++m) acc += U[k][m * ld + i] * cc[k * kMaxNu + m];
                        l[rr][k] -= acc;
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int k = 0; k < B; ++k)
                if (own(rr)) {
                    const int i = tid + rr * NT;
                    xaX[k * ldx + i] = (TX)l[rr][k];
                    if (chain) xbX[k * ldx + i] = act[k] ? (TX)T[k][kk * ld + i] : (TX)0;
                }
        __syncthreads();
        double hv[R][B], w[R][B];
        if (chain)
            spmm_rows<O, R, NT, B, TM, TX, true, true, true>(S, g, Hv, Sv, xaX, xbX, ldx, hv, w, zv);
        else
            spmm_rows<O, R, NT, B, TM, TX, true, true, false>(S, g, Hv, Sv, xaX, xbX, ldx, hv, w, dmy);
        group_sum<NWV, B>([&](double (&tt)[B]) __attribute__((always_inline)) {
#pragma unroll
            for (int k = 0; k < B; ++k) {
                double a = 0.0;
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
                    if (own(rr)) a += l[rr][k] * w[rr][k];
                tt[k] = a;
            }
        }, sm.scratch, gs);
        unsigned acc_mask = 0;
#pragma unroll
        for (int k = 0; k < B; ++k) {
            if (!act[k]) continue;
            const double bb = gs[k];
            double b0 = bb;
            for (int m = 0; m < cnt[k]; ++m) {
                const double cs = c1[k * kMaxNu + m] + c2[k * kMaxNu + m];
                b0 += cs * cs;
            }
            if (!(bb > 0.0) || !(b0 > 0.0) || sqrt(bb) <= J.tau * sqrt(b0)) continue;
            const double inv = 1.0 / sqrt(bb);
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int i = tid + rr * NT;
                if (i < n) {
                    U[k][L[k] * ld + i] = l[rr][k] * inv;
                    SU[k][L[k] * ld + i] = w[rr][k] * inv;
                    K[k][L[k] * ld + i] = hv[rr][k] * inv;
                }
                l[rr][k] = hv[rr][k] * inv;   // next block-1 seed: H u_L
            }
            ++L[k];
            acc_mask |= 1u << k;
        }
        return acc_mask;
    };

    bool act1[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
        act1[k] = status[k] == 0;
#pragma unroll
        for (int rr = 0; rr < R; ++rr) l[rr][k] = unit(rr, k);
    }
    // block 1: seeds e_j, H u_1, H u_2, ...
    for (int step = 0; step < J.p; ++step) {
        bool any = false;
#pragma unroll
        for (int k = 0; k < B; ++k) any |= act1[k];
        if (!any) break;
        const unsigned ok = append(act1, false, 0);
#pragma unroll
        for (int k = 0; k < B; ++k)
            if (act1[k] && !(ok & (1u << k))) act1[k] = false;
    }
    // block 2: chains t_1 = s_j / |s_j|, t_{k+1} = H t_k orthonormalised
    if (J.q > 0) {
        bool alive[B];
#pragma unroll
        for (int k = 0; k < B; ++k) alive[k] = status[k] == 0;
        for (int kk = 0; kk < J.q; ++kk) {
            bool any = false;
#pragma unroll
            for (int k = 0; k < B; ++k) any |= alive[k];
            if (!any) break;
#pragma unroll
            for (int k = 0; k < B; ++k)
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    const int i = tid + rr * NT;
                    l[rr][k] = (alive[k] && i < n) ? T[k][kk * ld + i] : 0.0;
                }
            const bool last = (kk + 1 == J.q);
            append(alive, !last, kk);
            if (last) break;
            // Euclidean Gram-Schmidt of H t_k against t_1..t_k, twice
            group_sum<NWV, B>([&](double (&tt)[B]) __attribute__((always_inline)) {
#pragma unroll
                for (int k = 0; k < B; ++k) {
                    double a = 0.0;
#pragma unroll
                    for (int rr = 0; rr < R; ++rr)
                        if (own(rr)) a += zv[rr][k] * zv[rr][k];
                    tt[k] = a;
                }
            }, sm.scratch, gs);
            double eta0[B];
#pragma unroll
            for (int k = 0; k < B; ++k) eta0[k] = sqrt(gs[k]);
            int cnt[B];
#pragma unroll
            for (int k = 0; k < B; ++k) cnt[k] = alive[k] ? kk + 1 : 0;
            for (int pass = 0; pass < 2; ++pass) {
                stage64(zv, sm.xb);
                __syncthreads();
                multidot_group<NWV, B>(T, ld, cnt, nb, sm.xb, ldx, n, c1);
                __syncthreads();
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    const int i = tid + rr * NT;
                    if (i < n) {
#pragma unroll
                        for (int k = 0; k < B; ++k) {
                            double acc = 0.0;
                            for (int m = 0; m < cnt[k]; ++m) acc += T[k][m * ld + i] * c1[k * kMaxNu + m];
                            zv[rr][k] -= acc;
                        }
                    }
                }
            }
            group_sum<NWV, B>([&](double (&tt)[B]) __attribute__((always_inline)) {
#pragma unroll
                for (int k = 0; k < B; ++k) {
                    double a = 0.0;
#pragma unroll
                    for (int rr = 0; rr < R; ++rr)
                        if (own(rr)) a += zv[rr][k] * zv[rr][k];
                    tt[k] = a;
                }
            }, sm.scratch, gs);
#pragma unroll
            for (int k = 0; k < B; ++k) {
                if (!alive[k]) continue;
                const double eta = sqrt(gs[k]);
                if (!(eta > J.tau * eta0[k])) {
                    alive[k] = false;
                    continue;
                }
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    const int i = tid + rr * NT;
                    if (i < n) T[k][(kk + 1) * ld + i] = zv[rr][k] / eta;
                }
            }
        }
    }
    __syncthreads();   // basis writes visible to the whole workgroup

    // ---------------- Galerkin pairs and basis rows, per column ----------------
    const int64_t kb0 = S.blk_ptr[A];
    const int npat = (int)(S.blk_ptr[A + 1] - kb0) * O;
    for (int k = 0; k < nb; ++k) {
        int Lk = 0, stk = 0, sk = 0, jk = 0;
        const double *Uk = U[0], *SUk = SU[0], *Kk = K[0];
#pragma unroll
        for (int kk = 0; kk < B; ++kk)
            if (kk == k) {
                Lk = L[kk];
                stk = status[kk];
                sk = slot[kk];
                jk = jl[kk];
                Uk = U[kk];
                SUk = SU[kk];
                Kk = K[kk];
            }
        if (stk != 0) continue;
        double *mid = J.mid + (int64_t)sk * J.mid_stride;
        double *Xh = mid, *Xs = mid + (int64_t)nu * nu;
        const int w = tid >> 6, lane = tid & 63;
        const int ntl = (Lk + 15) >> 4;
        for (int tile = w; tile < ntl * ntl; tile += NWV) {
            const int mt = tile / ntl, ntc = tile - mt * ntl;
            const int m = mt * 16 + (lane & 15), nn = ntc * 16 + (lane & 15);
            const int kq = lane >> 4;
            const bool mok = m < Lk, nok = nn < Lk;
            const double *um = Uk + (int64_t)(mok ? m : 0) * ld;
            const double *kn = Kk + (int64_t)(nok ? nn : 0) * ld;
            const double *sn = SUk + (int64_t)(nok ? nn : 0) * ld;
            dbl4 ah = {0.0, 0.0, 0.0, 0.0}, as = {0.0, 0.0, 0.0, 0.0};
            for (int i0 = 0; i0 < n; i0 += 4) {
                const int i = i0 + kq;
                const bool iok = i < n;
                const double a = (mok && iok) ? um[i] : 0.0;
                const double bh = (nok && iok) ? kn[i] : 0.0;
                const double bs = (nok && iok) ? sn[i] : 0.0;
                ah = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bh, ah, 0, 0, 0);
                as = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bs, as, 0, 0, 0);
            }
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const int mr = mt * 16 + 4 * jj + kq, nc = ntc * 16 + (lane & 15);
                if (mr < Lk && nc < Lk) {
                    Xh[mr * nu + nc] = ah[jj];
                    Xs[mr * nu + nc] = as[jj];
                }
            }
        }
        double *Up = mid + 2 * (int64_t)nu * nu;
        for (int e = tid; e < (npat + 2) * Lk; e += NT) {
            const int row = e / Lk, m = e - row * Lk;
            double v;
            if (row == 0) v = Uk[m * ld + jk];
            else if (row == 1) v = SUk[m * ld + jk];
            else {
                const int tt = row - 2;
                v = Uk[m * ld + S.blk_loc[kb0 + tt / O] * O + (tt % O)];
            }
            Up[row * nu + m] = v;
        }
    }
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < B; ++k)
            if (valid(k)) write_stats(J, cc_[k], L[k], iters[k], nres[k], status[k], start[k]);
    }
    __syncthreads();
}

template <int O, int B, int NT, int R, int PREC>
__global__ void __launch_bounds__(NT) k_basis_m(DevSystem S, DevJob J)
{
    extern __shared__ double smem[];
    __shared__ int s_idx;
    __shared__ double gsum[16];
    SmemM sm;
    sm.ldx = S.nmax;
    sm.xa = smem;
    sm.xb = smem + B * S.nmax;
    sm.cf = smem + 2 * B * S.nmax;
    sm.scratch = sm.cf + 2 * B * kMaxNu;
    sm.gs = gsum;
    double *ws = J.ws + (int64_t)blockIdx.x * J.ws_stride;
    drain_queues_raw(J, &s_idx, [&](int idx) __attribute__((always_inline)) {
        basis_group<O, B, NT, R, PREC>(S, J, sm, idx, ws);
    });
}

// ------------------------------------------------------------------------
// small-region basis kernel: basis on chip
// ------------------------------------------------------------------------
// Thread t owns local row t (n <= NT).  U[m] lives in LDS (row stride
// nmax), S u_m and the chain vectors t_k in the thread's registers, so every
// access to the basis is to the thread's own row.  The S-orthogonalisation is
// the delayed two-pass classical Gram-Schmidt of the workspace kernel (one
// reduction per basis vector); the Galerkin pair is accumulated as each
// vector's S and H images become available: X[m][L] = u_m^T H u_L (upper
// triangle, mirrored), S~[m][L] = u_m^T (S u_L) and S~[L][m] = u_L^T (S u_m).
// Each step reduces one set of per-row partial products over the workgroup
// (transposed wavefront reductions, then the wavefront totals in LDS).
template <int O, int NT, int NU, int PREC>
__device__ void basis_small(const DevSystem &S, const DevJob &J, double *Ub, double *xa,
                            double *xb, double *xz, double *scratch, double *rs, double *cf,
                            int *srp, int2 *sblk, double *red, float *redf, int c, int s)
{
    using TM = typename std::conditional<PREC != 0, float, double>::type;
    using TX = typename std::conditional<PREC == 1, float, double>::type;
    constexpr int NWV = NT / 64;
    constexpr int NQ = NU / 2;
    constexpr int G = 7;   // reduction groups of NU values, see below
    const int o = O ? O : S.o;
    const int tid = threadIdx.x;
    const int ldu = S.nmax;
    const int nu = J.nu;
    Col g = make_col(S, J, c, o);
    if (J.lidx) stage_col_index<NT>(S, g, srp, sblk);
    const int n = g.n;
    const bool own = tid < n;
    const TM *Hv = PREC ? (const TM *)S.Hf : (const TM *)S.Hd;
    const TM *Sv = PREC ? (const TM *)S.Sf : (const TM *)S.Sd;
    TX *xaX = reinterpret_cast<TX *>(xa);
    TX *xbX = reinterpret_cast<TX *>(xb);
    TX *xzX = reinterpret_cast<TX *>(xz);

    double x[1];
    int iters, nres, status, start;
    inner_cg<O, 1, NT, PREC>(S, J, g, c, xa, xb, red, redf, x, iters, nres, status, start);

    double *mid = J.mid + (int64_t)s * J.mid_stride;
    double *Xh = mid, *Xs = mid + (int64_t)nu * nu, *Up = mid + 2 * (int64_t)nu * nu;
    double SU[NU];   // (S u_m) at this thread's row
    double Tc[NQ];   // chain vector t_k at this thread's row
#pragma unroll
    for (int m = 0; m < NU; ++m) SU[m] = 0.0;
#pragma unroll
    for (int m = 0; m < NQ; ++m) Tc[m] = 0.0;
    int L = 0;
    if (status == 0) {
        double *cbuf0 = cf, *cbuf1 = cf + (NU + 1), *ctb0 = cf + 2 * (NU + 1), *ctb1 = ctb0 + (NQ + 1);
        // own-row state: uf finished vector (images pending), p pending
        // vector, zt pending chain vector
        double uf = 0.0, p = (tid == g.jl) ? 1.0 : 0.0, zt = own ? x[0] : 0.0;
        bool has_fin = false, has_pend = J.p > 0;
        bool b1_live = true, chain_live = J.q > 0;
        int nb1 = J.p > 0 ? 1 : 0, k = 0, ping = 0;
        double cp_scale = 1.0, ctp_scale = 1.0;
        __syncthreads();   // the CG's last reads of xa, xb are done
        if (own) {
            xaX[tid] = (TX)0.0;
            xbX[tid] = (TX)p;
            xzX[tid] = (TX)zt;
        }
        for (;;) {
            const int kind = (b1_live && nb1 < J.p) ? kCandBlock1
                             : chain_live ? kCandChain : kCandNone;
            if (!has_fin && !has_pend && kind == kCandNone) break;
            const bool need_z = kind == kCandChain && k + 1 < J.q;
            const TX *xd = kind == kCandChain ? xzX : xbX;
            double *cp = ping ? cbuf0 : cbuf1, *cbn = ping ? cbuf1 : cbuf0;
            double *ctp = ping ? ctb0 : ctb1, *ctn = ping ? ctb1 : ctb0;

            // ---- SpMV ----
            __syncthreads();   // staged vectors visible
            double hf1[1], sf1[1], sp1[1], hz1[1];
            spmv3_rows<O, 1, NT, TM, TX>(S, g, o, Hv, Sv, xaX, xbX, xd, hf1, sf1, sp1, hz1);
            const double hf = hf1[0], sf = sf1[0], sp = sp1[0], hz = hz1[0];
            if (has_fin) {
#pragma unroll
                for (int m = 0; m < NU; ++m) SU[m] = (m == L - 1) ? sf : SU[m];
            }
            const bool tail = kind == kCandNone && !has_pend;
            const double cand = kind == kCandChain ? zt : hz;

            // ---- one reduction: dots, Galerkin column L-1, scalars ----
            // groups: 0 a = (S U)^T p, 1 b = (S U)^T candidate,
            // 2 [T^T zt | T^T H zt], 3 U^T H u_{L-1}, 4 U^T S u_{L-1},
            // 5 (S U)^T u_{L-1}, 6 scalars
            block_reduce<NWV, NU, G>([&](int gi, double (&v)[NU]) __attribute__((always_inline)) {
#pragma unroll
                for (int m = 0; m < NU; ++m) {
                    double val = 0.0;
                    if (own) {
                        if (gi == 0) val = (m < L && !tail) ? SU[m] * p : 0.0;
                        else if (gi == 1) val = (m < L && !tail) ? SU[m] * cand : 0.0;
                        else if (gi == 2) {
                            if (kind == kCandChain) {
                                if (m < NQ) val = m < k ? Tc[m & (NQ - 1)] * zt : 0.0;
                                else val = (m - NQ) < k ? Tc[(m - NQ) & (NQ - 1)] * hz : 0.0;
                            }
                        } else if (gi == 3 || gi == 4) {
                            const double um = (has_fin && m < L) ? Ub[m * ldu + tid] : 0.0;
                            val = um * (gi == 3 ? hf : sf);
                        } else if (gi == 5) {
                            val = (has_fin && m < L) ? uf * SU[m] : 0.0;
                        } else {
                            val = m == 0 ? p * sp : m == 1 ? sp * cand : m == 2 ? zt * zt
                                  : m == 3 ? zt * hz : 0.0;
                        }
                    }
                    v[m] = val;
                }
            }, scratch, rs);
            const double *ca = rs, *cb = rs + NU, *cat = rs + 2 * NU, *ctb = rs + 2 * NU + NQ;
            if (has_fin) {
                // Galerkin column L-1
                for (int m = tid; m < L; m += NT) {
                    const double h = rs[3 * NU + m];
                    Xh[m * nu + (L - 1)] = h;
                    Xh[(L - 1) * nu + m] = h;
                    Xs[m * nu + (L - 1)] = rs[4 * NU + m];
                    if (m < L - 1) Xs[(L - 1) * nu + m] = rs[5 * NU + m];
                }
            }
            if (tail) break;
            const double nu_p = rs[6 * NU + 0], e_p = rs[6 * NU + 1];
            const double nu_t = rs[6 * NU + 2], e_t = rs[6 * NU + 3];

            // ---- decisions (every thread, same values) ----
            bool acc_u = false;
            double beta = 1.0, f = 0.0;
            if (has_pend) {
                double asq = 0.0, tot = 0.0, ab = 0.0;
                for (int m = 0; m < L; ++m) {
                    const double cm = cp_scale * cp[m] + ca[m];
                    asq += ca[m] * ca[m];
                    tot += cm * cm;
                    if (kind != kCandNone) ab += ca[m] * cb[m];
                }
                const double bb = nu_p - asq, b0 = bb + tot;
                acc_u = bb > 0.0 && b0 > 0.0 && !(sqrt(bb) <= J.tau * sqrt(b0));
                if (acc_u) {
                    beta = sqrt(bb);
                    f = (e_p - ab) / beta;
                }
            }
            bool acc_t = false;
            double eta = 1.0, ft = 0.0;
            if (kind == kCandChain) {
                double asq = 0.0, tot = 0.0, ab = 0.0;
                for (int m = 0; m < k; ++m) {
                    const double cm = ctp_scale * ctp[m] + cat[m];
                    asq += cat[m] * cat[m];
                    tot += cm * cm;
                    ab += cat[m] * ctb[m];
                }
                const double ee = nu_t - asq, e0 = ee + tot;
                acc_t = ee > 0.0 && sqrt(ee) > J.tau * sqrt(e0);
                if (acc_t) {
                    eta = sqrt(ee);
                    ft = (e_t - ab) / eta;
                }
            }
            const bool new_pend = (kind == kCandBlock1 && acc_u) || (kind == kCandChain && acc_t);
            const bool new_chain = need_z && acc_t;
            const double inv_b = 1.0 / beta, inv_e = 1.0 / eta;
            const double sc = kind == kCandBlock1 ? inv_b : 1.0;
            // first-pass coefficients of the new pending vectors, kept for the next step
            for (int m = tid; m < L; m += NT) cbn[m] = cb[m];
            for (int m = tid; m < k; m += NT) ctn[m] = ctb[m];
            if (tid == 0) {
                if (acc_u) cbn[L] = f;
                if (acc_t) ctn[k] = ft;
            }

            // ---- update of the thread's row ----
            if (own) {
                double sa = 0.0, sb = 0.0;
                if (acc_u || new_pend) {
#pragma unroll 8
                    for (int m = 0; m < L; ++m) {
                        const double um = Ub[m * ldu + tid];
                        sa += um * ca[m];
                        sb += um * cb[m];
                    }
                }
                double ta = 0.0, tb = 0.0;
#pragma unroll
                for (int m = 0; m < NQ; ++m) {
                    if (m < k) {
                        ta += Tc[m] * cat[m];
                        tb += Tc[m] * ctb[m];
                    }
                }
                const double u = (p - sa) * inv_b;
                const double nl = (cand - sb - (acc_u ? f * u : 0.0)) * sc;
                const double t = (zt - ta) * inv_e;
                const double nz = (hz - tb - ft * t) * inv_e;
                if (acc_u) {
                    Ub[L * ldu + tid] = u;
                    xaX[tid] = (TX)u;
                    uf = u;
                }
                if (acc_t) {
#pragma unroll
                    for (int m = 0; m < NQ; ++m) Tc[m] = (m == k) ? t : Tc[m];
                }
                p = new_pend ? nl : 0.0;
                xbX[tid] = (TX)p;
                if (new_chain) {
                    zt = nz;
                    xzX[tid] = (TX)zt;
                }
            }
            if (kind == kCandBlock1) {
                if (acc_u) ++nb1;
                else b1_live = false;
            }
            if (kind == kCandChain) {
                if (acc_t) {
                    ++k;
                    chain_live = k < J.q;
                } else {
                    chain_live = false;
                }
            }
            if (acc_u) ++L;
            cp_scale = sc;
            ctp_scale = inv_e;
            has_fin = acc_u;
            has_pend = new_pend;
            ping ^= 1;
        }
        __syncthreads();   // U complete in LDS

        // rows of U the outputs need: u at row j, S u at row j, u at the pattern rows
        const int64_t kb0 = S.blk_ptr[g.A];
        const int npat = (int)(S.blk_ptr[g.A + 1] - kb0) * o;
        for (int e = tid; e < (npat + 1) * L; e += NT) {
            const int rr = e / L, m = e - rr * L;
            int i, row;
            if (rr == 0) {
                i = g.jl;
                row = 0;
            } else {
                const int tt = rr - 1;
                i = S.blk_loc[kb0 + tt / o] * o + (tt % o);
                row = tt + 2;
            }
            Up[row * nu + m] = Ub[m * ldu + i];
        }
        if (tid == g.jl) {
#pragma unroll
            for (int m = 0; m < NU; ++m)
                if (m < L) Up[nu + m] = SU[m];
        }
    }
    if (tid == 0) write_stats(J, c, L, iters, nres, status, start);
    __syncthreads();   // U, the staged vectors and the index are reused by the next column
}

// LDS of the on-chip kernel in doubles, besides U (nu * nmax) and the index:
// three staged vectors, the reduction scratch and results, coefficients
template <int NT, int NU>
__host__ __device__ constexpr int small_smem_doubles_fixed()
{
    return (NT / 64) * 7 * NU + 7 * NU + 2 * (NU + 1) + 2 * (NU / 2 + 1);
}

template <int O, int NT, int NU, int PREC>
__global__ void __launch_bounds__(NT) k_basis_s(DevSystem S, DevJob J)
{
    extern __shared__ double smem[];
    __shared__ double red[NT / 64];
    __shared__ float redf[NT / 64];
    __shared__ int s_idx;
    double *Ub = smem;
    double *xa = Ub + (int64_t)J.nu * S.nmax;
    double *xb = xa + S.nmax;
    double *xz = xb + S.nmax;
    double *scratch = xz + S.nmax;
    double *rs = scratch + (NT / 64) * 7 * NU;
    double *cf = rs + 7 * NU;
    int *srp = reinterpret_cast<int *>(cf + 2 * (NU + 1) + 2 * (NU / 2 + 1));
    int2 *sblk = reinterpret_cast<int2 *>(srp + ((S.max_nat + 2) & ~1));
    drain_queues(J, &s_idx, [&](int c, int s) __attribute__((always_inline)) {
        basis_small<O, NT, NU, PREC>(S, J, Ub, xa, xb, xz, scratch, rs, cf, srp, sblk, red, redf,
                                     c, s);
    });
}

// ------------------------------------------------------------------------
// reduced generalised eigenproblems and column outputs (a6, a7)
// ------------------------------------------------------------------------
// One wavefront per column of the chunk, everything in LDS:
//   1/2 (X + X^T) -> H~, S~; Cholesky S~ = Lc Lc^T (right-looking);
//   A = Lc^-1 H~ Lc^-T (two right-looking triangular solves, a lane per column);
//   Householder reduction A = Q T Q^T to tridiagonal T, Q accumulated backwards;
//   implicit QL iterations with shifts on T (the published QL algorithm for
//   symmetric tridiagonal matrices: Bowdler, Martin, Reinsch and Wilkinson,
//   Numer. Math. 11 (1968)), each plane rotation applied to the rows of Z = Q
//   by one lane per row;
//   C = Lc^-T Z.
// Every lane runs the scalar recurrences of the QL sweeps redundantly, so they
// need no broadcasts.  Then v_a at row j, (S v_a)_j, the Ritz values in
// ascending order and the weights w_a = v_ja (S v_a)_j; then either the
// amplitudes v_ia v_ja at the pattern rows or, with a given chemical
// potential, rho_ij, pi_ij (Eqs. 13-14) and E_j, N_j (Eq. 17).
template <typename TA>
__global__ void __launch_bounds__(64) k_eig(DevSystem S, DevJob J)
{
    extern __shared__ double smem[];
    const int nu = J.nu;
    // Two nu x nu matrices in LDS (A, and Z column-major); the Cholesky
    // factor of S~ lives in the Z area until Z is needed, waits in the S~
    // slot of the chunk buffer meanwhile, and comes back for C = Lc^-T Z.
    double *A = smem, *Z = smem + nu * nu, *B = Z;
    double *ev = smem + 2 * nu * nu, *vj = ev + nu, *svj = vj + nu, *fw = svj + nu;
    double *hh = fw + nu, *ee = hh + nu, *rd = ee + nu;
    double *upj = rd + nu;   // 2 nu
    int *rank = reinterpret_cast<int *>(upj + 2 * nu);
    int *inv = rank + nu;
    __shared__ double hv[kMaxNu];   // current Householder vector (separate objects: the
    __shared__ double hq[kMaxNu];   // compiler may keep their loads ahead of A's stores)
    const int lane = threadIdx.x;
    const int o = S.o;
    for (int s = blockIdx.x; s < J.cn; s += gridDim.x) {
        const int c = J.order[J.c0 + s];
        double *mid = J.mid + (int64_t)s * J.mid_stride;
        const double *Up = mid + 2 * (int64_t)nu * nu;
        int32_t *st = J.stats + (int64_t)c * kStats;
        int L = st[3] == 0 ? st[0] : 0;
        int status = 0;
#pragma unroll 4
        for (int e = lane; e < L * L; e += 64) {
            const int i = e / L, k = e - i * L;
            A[e] = 0.5 * (mid[i * nu + k] + mid[k * nu + i]);
            B[e] = 0.5 * (mid[nu * nu + i * nu + k] + mid[nu * nu + k * nu + i]);
        }
        // basis rows at j: u_m[j] and (S u_m)[j]
        for (int m = lane; m < L; m += 64) {
            upj[m] = Up[m];
            upj[nu + m] = Up[nu + m];
        }
        __syncthreads();

        // Cholesky S~ = Lc Lc^T in the lower triangle of B
        for (int k = 0; k < L; ++k) {
            double dk = B[k * L + k];
            if (!(dk > 0.0)) {
                status = -4;
                dk = 1.0;
            }
            const double lk = sqrt(dk), rl = 1.0 / lk;
            for (int i = k + 1 + lane; i < L; i += 64) B[i * L + k] *= rl;
            __syncthreads();
            for (int j = k + 1 + lane; j < L; j += 64) {
                const double bjk = B[j * L + k];
                #pragma unroll 4
                for (int i = j; i < L; ++i) B[i * L + j] -= B[i * L + k] * bjk;
            }
            if (lane == 0) {
                B[k * L + k] = lk;
                rd[k] = rl;
            }
            __syncthreads();
        }
        // A = Lc^-1 H~ Lc^-T in place: W = Lc^-1 A (a lane per column), then
        // A = Lc^-1 W^T
        for (int pass = 0; pass < 2; ++pass) {
            for (int k = 0; k < L; ++k)
                for (int cc = lane; cc < L; cc += 64) {
                    const double ak = A[k * L + cc] * rd[k];
                    A[k * L + cc] = ak;
                    #pragma unroll 4
                    for (int i = k + 1; i < L; ++i) A[i * L + cc] -= B[i * L + k] * ak;
                }
            __syncthreads();
            if (pass == 0) {
                for (int e = lane; e < L * L; e += 64) {
                    const int i = e / L, k = e - i * L;
                    if (i < k) {
                        const double x = A[i * L + k];
                        A[i * L + k] = A[k * L + i];
                        A[k * L + i] = x;
                    }
                }
                __syncthreads();
            }
        }
        // the factor waits in the S~ slot of the chunk buffer (read above,
        // not read again) while Z takes its place
        for (int e = lane; e < L * L; e += 64) mid[nu * nu + e] = B[e];
        __syncthreads();
        for (int e = lane; e < L * L; e += 64) {
            const int i = e / L, k = e - i * L;
            if (i < k) {
                const double v = 0.5 * (A[i * L + k] + A[k * L + i]);
                A[i * L + k] = v;
                A[k * L + i] = v;
            }
        }
        __syncthreads();

        // Householder reduction to tridiagonal form.  Step k reflects
        // x = A[k+1.., k] onto alpha e_1 with P = I - v v^T / h,
        // v = x - alpha e_1, h = |v|^2 / 2; v stays in column k below the
        // diagonal, h in hh[k], alpha is the sub-diagonal ee[k].
        for (int k = 0; k + 2 < L; ++k) {
            const int i = k + 1 + lane;
            const double xi = i < L ? A[i * L + k] : 0.0;
            const double sig = wave_sum(xi * xi);
            const double x0 = A[(k + 1) * L + k];
            double alpha = x0, h = 0.0;
            if (sig > 0.0) {
                alpha = x0 >= 0.0 ? -sqrt(sig) : sqrt(sig);
                h = sig - x0 * alpha;
            }
            if (lane == 0) {
                ee[k] = alpha;
                hh[k] = h;
            }
            if (h > 0.0) {
                // v = x - alpha e_1, kept in column k and in hv
                const double vi = (i == k + 1) ? x0 - alpha : xi;
                if (i < L) {
                    hv[i] = vi;
                    A[i * L + k] = vi;
                }
                __syncthreads();
                // p = A' v / h, K = v^T p / (2 h), q = p - K v (a lane per column j)
                const int j = k + 1 + lane;
                double pj = 0.0, vjj = 0.0;
                if (j < L) {
                    #pragma unroll 4
                    for (int ii = k + 1; ii < L; ++ii) pj += A[ii * L + j] * hv[ii];
                    pj /= h;
                    vjj = hv[j];
                }
                const double K = wave_sum(vjj * pj) / (2.0 * h);
                const double qj = pj - K * vjj;
                if (j < L) hq[j] = qj;
                __syncthreads();
                // A' -= v q^T + q v^T
                if (j < L)
                    #pragma unroll 4
                    for (int ii = k + 1; ii < L; ++ii)
                        A[ii * L + j] -= hv[ii] * qj + hq[ii] * vjj;
            }
            __syncthreads();
        }
        for (int i = lane; i < L; i += 64) ev[i] = A[i * L + i];
        if (lane == 0 && L >= 2) ee[L - 2] = A[(L - 1) * L + L - 2];
        if (lane == 0 && L >= 1) ee[L - 1] = 0.0;
        // Z = P_0 P_1 ... P_{L-3} (column-major), accumulated from the last
        // reflector; P_k leaves columns 0..k unchanged
        for (int e = lane; e < L * L; e += 64) Z[e] = (e / L == e % L) ? 1.0 : 0.0;
        __syncthreads();
        for (int k = L - 3; k >= 0; --k) {
            const double h = hh[k];
            if (!(h > 0.0)) continue;
            for (int cc = k + 1 + lane; cc < L; cc += 64) {
                double t = 0.0;
                #pragma unroll 4
                for (int i = k + 1; i < L; ++i) t += A[i * L + k] * Z[cc * L + i];
                t /= h;
                #pragma unroll 4
                for (int i = k + 1; i < L; ++i) Z[cc * L + i] -= A[i * L + k] * t;
            }
        }
        __syncthreads();

        // Implicit QL sweeps on (ev, ee).  For the leading unreduced block
        // [l, m] (ee[m] negligible against its diagonal neighbours), a shift
        // from the 2 x 2 at l, then plane rotations chasing the bulge from m
        // up to l.  At most 64 sweeps per eigenvalue.  The rotation loop is
        // software-pipelined: the entries of the next rotation are loaded one
        // rotation ahead, and the rotated column i stays in a register for the
        // next rotation (columns i + 1 are final once written).
        for (int l = 0; l < L && status == 0; ++l) {
            int sweeps = 0;
            for (;;) {
                // m: the first k >= l with ee[k] negligible (L - 1 if none),
                // one lane per k
                bool small = lane == L - 1;
                if (lane >= l && lane < L - 1)
                    small = fabs(ee[lane]) <= DBL_EPSILON * (fabs(ev[lane]) + fabs(ev[lane + 1]));
                const unsigned long long msk =
                    __ballot(small) & ~((l > 0 ? (1ull << l) : 1ull) - 1ull);
                const int m = __ffsll((long long)msk) - 1;
                if (m == l) break;
                if (++sweeps > 64) {
                    status = -5;
                    break;
                }
                const double el = ee[l], dl0 = ev[l], dl1 = ev[l + 1], dm = ev[m];
                const double t0 = (dl1 - dl0) / (2.0 * el);
                const double r0 = sqrt(t0 * t0 + 1.0);
                double g = dm - dl0 + el / (t0 + (t0 >= 0.0 ? r0 : -r0));
                double sn = 1.0, cs = 1.0, p = 0.0;
                bool underflow = false;
                const bool row = lane < L;
                double e_i = ee[m - 1], d_i = ev[m - 1], d_i1 = dm;
                double z_i1 = row ? Z[m * L + lane] : 0.0;
                double z_i = row ? Z[(m - 1) * L + lane] : 0.0;
                for (int i = m - 1; i >= l; --i) {
                    double e_n = 0.0, d_n = 0.0, z_n = 0.0;
                    if (i > l) {
                        e_n = ee[i - 1];
                        d_n = ev[i - 1];
                        z_n = row ? Z[(i - 1) * L + lane] : 0.0;
                    }
                    const double f = sn * e_i, b = cs * e_i;
                    const double r2 = f * f + g * g;
                    if (r2 == 0.0) {
                        const double dnew = d_i1 - p;
                        if (lane == 0) {
                            ee[i + 1] = 0.0;
                            ev[i + 1] = dnew;
                            ee[m] = 0.0;
                        }
                        if (row) Z[(i + 1) * L + lane] = z_i1;
                        underflow = true;
                        break;
                    }
                    const double ir = rsqrt(r2);
                    sn = f * ir;
                    cs = g * ir;
                    g = d_i1 - p;
                    const double rr = (d_i - g) * sn + 2.0 * cs * b;
                    p = sn * rr;
                    if (lane == 0) {
                        ee[i + 1] = r2 * ir;
                        ev[i + 1] = g + p;
                    }
                    g = cs * rr - b;
                    const double zn1 = sn * z_i + cs * z_i1;
                    const double zn0 = cs * z_i - sn * z_i1;
                    if (row) Z[(i + 1) * L + lane] = zn1;
                    z_i1 = zn0;
                    z_i = z_n;
                    e_i = e_n;
                    d_i1 = d_i;
                    d_i = d_n;
                }
                if (underflow) continue;
                if (row) Z[l * L + lane] = z_i1;
                if (lane == 0) {
                    ev[l] = dl0 - p;
                    ee[l] = g;
                    ee[m] = 0.0;
                }
            }
        }
        __syncthreads();
        // ascending ranks of the eigenvalues
        for (int a = lane; a < L; a += 64) {
            int rk = 0;
            const double va = ev[a];
            #pragma unroll 4
            for (int bb = 0; bb < L; ++bb)
                if (ev[bb] < va || (ev[bb] == va && bb < a)) ++rk;
            rank[a] = rk;
        }
        // C = Lc^-T Z -> A (row-major), a lane per column; the factor back
        // in the Z area once Z is copied
        for (int a = lane; a < L; a += 64) {
            #pragma unroll 4
            for (int i = 0; i < L; ++i) A[i * L + a] = Z[a * L + i];
        }
        __syncthreads();
        for (int e = lane; e < L * L; e += 64) B[e] = mid[nu * nu + e];
        __syncthreads();
        for (int a = lane; a < L; a += 64) {
            for (int k = L - 1; k >= 0; --k) {
                const double ck = A[k * L + a] * rd[k];
                A[k * L + a] = ck;
                #pragma unroll 4
                for (int i = 0; i < k; ++i) A[i * L + a] -= B[k * L + i] * ck;
            }
        }
        __syncthreads();
        if (status != 0) {
            L = 0;
            if (lane == 0) {
                st[0] = 0;
                st[3] = status;
                atomicMin(J.fail, c);
            }
        }
        const double *C = A;
        // v_a and (S v_a) at row j (a lane per Ritz vector; the basis rows
        // are read at the same address by every lane)
        for (int a = lane; a < L; a += 64) {
            double v1 = 0.0, v2 = 0.0;
            #pragma unroll 4
            for (int m = 0; m < L; ++m) {
                const double cma = C[m * L + a];
                v1 += upj[m] * cma;
                v2 += upj[nu + m] * cma;
            }
            vj[a] = v1;
            svj[a] = v2;
        }
        __syncthreads();
        double *eps_o = J.eps + (int64_t)c * nu, *wts_o = J.wts + (int64_t)c * nu;
        for (int a = lane; a < nu; a += 64) {
            if (a < L) {
                eps_o[rank[a]] = ev[a];
                wts_o[rank[a]] = vj[a] * svj[a];
                inv[rank[a]] = a;
            } else {
                eps_o[a] = NAN;
                wts_o[a] = 0.0;
            }
        }
        const int j = J.cols[c];
        const int At = j / o, r = j - At * o;
        const int64_t kb0 = S.blk_ptr[At];
        const int npat = (int)(S.blk_ptr[At + 1] - kb0) * o;
        if (!J.direct) {
            // V at the pattern rows on the FP64 matrix cores: 16 x 16 tiles of
            // (basis rows of the chunk buffer, npat x L) x (C, L x L, LDS), with
            // v_mfma_f64_16x16x4f64: lane l feeds A[l%16][l/16], B[l/16][l%16]
            // and receives D[4 j + l/16][l%16]
            TA *amp = reinterpret_cast<TA *>(J.amp) + J.amp_off[c];
            const int nrt = (npat + 15) >> 4, nct = (nu + 15) >> 4;
            const int kq = lane >> 4, l16 = lane & 15;
            for (int mt = 0; mt < nrt; ++mt) {
                const int arow = mt * 16 + l16;
                // this lane's basis-row operands for the first 32 k, loaded together
                double avs[8];
#pragma unroll
                for (int st4 = 0; st4 < 8; ++st4) {
                    const int kk = 4 * st4 + kq;
                    avs[st4] = (arow < npat && kk < L) ? Up[(2 + arow) * nu + kk] : 0.0;
                }
              for (int ct = 0; ct < nct; ++ct) {
                const int bcol = ct * 16 + l16;
                dbl4 acc = {0.0, 0.0, 0.0, 0.0};
                for (int k0 = 0; k0 < L; k0 += 4) {
                    const int kk = k0 + kq;
                    const double av = k0 < 32 ? avs[(k0 >> 2) & 7]
                                      : (arow < npat && kk < L) ? Up[(2 + arow) * nu + kk] : 0.0;
                    const double bv = (bcol < L && kk < L) ? C[kk * L + bcol] : 0.0;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int tr = mt * 16 + 4 * jj + kq;
                    if (tr < npat && bcol < nu) {
                        if (bcol < L) amp[tr * nu + rank[bcol]] = (TA)(acc[jj] * vj[bcol]);
                        else amp[tr * nu + bcol] = (TA)0.0;
                    }
                }
              }
            }
        } else {
            __syncthreads();
            for (int k = lane; k < L; k += 64) fw[k] = fermi((ev[inv[k]] - J.mu) / J.kT);
            __syncthreads();
            double ep = 0.0, np_ = 0.0;
            for (int tt = lane; tt < npat; tt += 64) {
                double sr = 0.0, sp = 0.0;
                for (int k = 0; k < L; ++k) {
                    const int a = inv[k];
                    double v = 0.0;
                    #pragma unroll 4
                    for (int m = 0; m < L; ++m) v += Up[(2 + tt) * nu + m] * C[m * L + a];
                    const double am = v * vj[a];
                    sr += fw[k] * am;
                    sp += (fw[k] * ev[a]) * am;
                }
                const int64_t slot = ((kb0 + tt / o) * o + r) * o + (tt % o);
                if (J.rho) J.rho[slot] = sr;
                if (J.pi) J.pi[slot] = sp;
                ep += sr * S.Hd[slot];
                np_ += sr * S.Sd[slot];
            }
            ep = wave_sum(ep);
            np_ = wave_sum(np_);
            if (lane == 0) {
                J.Ecol[c] = ep;
                J.Ncol[c] = np_;
            }
        }
        __syncthreads();   // LDS is reused by the next column
    }
}

__global__ void k_reset(int *queue, int *fail, int reset_fail)
{
    for (int k = 0; k < kMaxQueues; ++k) queue[k] = 0;
    if (reset_fail) fail[0] = INT_MAX;
}

// ------------------------------------------------------------------------
// Fermi weighting and the chemical potential
// ------------------------------------------------------------------------
// Bracket of the chemical potential: [min eps - 50 kT, max eps + 50 kT] over
// the accepted Ritz values.  Per-block extremes, then one block combines them.
__global__ void __launch_bounds__(256) k_minmax(const double *eps, const int32_t *stats, int ncols,
                                                int nu, double *part)
{
    __shared__ double smin[4], smax[4];
    double lo = INFINITY, hi = -INFINITY;
    const int64_t total = (int64_t)ncols * nu;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / nu;
        if (e - c * nu < stats[c * kStats]) {
            lo = fmin(lo, eps[e]);
            hi = fmax(hi, eps[e]);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        smin[threadIdx.x >> 6] = lo;
        smax[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 4; ++k) {
            lo = fmin(lo, smin[k]);
            hi = fmax(hi, smax[k]);
        }
        lo = fmin(lo, smin[0]);
        hi = fmax(hi, smax[0]);
        part[2 * blockIdx.x] = lo;
        part[2 * blockIdx.x + 1] = hi;
    }
}

__global__ void __launch_bounds__(64) k_minmax_final(const double *part, int nblocks, double kT,
                                                     double *lohi, unsigned *done)
{
    double lo = INFINITY, hi = -INFINITY;
    for (int b = threadIdx.x; b < nblocks; b += 64) {
        lo = fmin(lo, part[2 * b]);
        hi = fmax(hi, part[2 * b + 1]);
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    if (threadIdx.x == 0) {
        lohi[0] = lo - 50.0 * kT;
        lohi[1] = hi + 50.0 * kT;
        *done = 0u;   // the K-section passes' completion counter
    }
}

// completion counter of the K-section passes: the word after the partial sums
__host__ __device__ inline unsigned *count_done(double *partial)
{
    return reinterpret_cast<unsigned *>(partial + kCountBlocks * kBisectTrials);
}

// Electron count sum_j sum_a f((eps_a - mu_t)/kT) w_a for the kBisectTrials
// trial potentials mu_t equally spaced inside (lo, hi); one partial per block.
// One K-section pass: every block evaluates the electron count at KT_
// equally spaced trial potentials over its share of the Ritz pairs and
// writes its partial sums; the last block to finish (a device-scope counter)
// sums the partials of all blocks in a fixed order and narrows the bracket
// to the first trial whose count reaches the target, then clears the
// counter for the next pass.
__global__ void __launch_bounds__(256) k_count(const double *eps, const double *wts,
                                               const int32_t *stats, int ncols, int nu,
                                               double kT, double n_target, double *lohi,
                                               double *partial, unsigned *done)
{
    constexpr int KT_ = kBisectTrials;
    __shared__ double sred[4][KT_];
    __shared__ int last;
    const double lo = lohi[0], hi = lohi[1];
    double acc[KT_];
#pragma unroll
    for (int t = 0; t < KT_; ++t) acc[t] = 0.0;
    const int64_t total = (int64_t)ncols * nu;
    const int64_t chunk = (total + gridDim.x - 1) / gridDim.x;
    const int64_t e0 = blockIdx.x * chunk, e1 = min(total, e0 + chunk);
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const int64_t c = e / nu;
        if (e - c * nu >= stats[c * kStats]) continue;
        const double ev = eps[e], w = wts[e];
#pragma unroll
        for (int t = 0; t < KT_; ++t) {
            const double mu = lo + (hi - lo) * (double)(t + 1) / (double)(KT_ + 1);
            acc[t] += fermi((ev - mu) / kT) * w;
        }
    }
#pragma unroll
    for (int t = 0; t < KT_; ++t) {
        const double v = wave_sum(acc[t]);
        if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6][t] = v;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < KT_; t += blockDim.x)
        partial[blockIdx.x * KT_ + t] = ((sred[0][t] + sred[1][t]) + sred[2][t]) + sred[3][t];
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(done, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    // fixed order: thread b adds blocks b, b + 256, ...; then wavefronts, then waves 0..3
#pragma unroll
    for (int t = 0; t < KT_; ++t) acc[t] = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x)
#pragma unroll
        for (int t = 0; t < KT_; ++t) acc[t] += __builtin_nontemporal_load(partial + b * KT_ + t);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < KT_; ++t) {
        const double v = wave_sum(acc[t]);
        if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6][t] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int first = KT_;
        for (int t = 0; t < KT_; ++t)
            if (((sred[0][t] + sred[1][t]) + sred[2][t]) + sred[3][t] >= n_target) {
                first = t;
                break;
            }
        const double nlo = first == 0 ? lo : lo + (hi - lo) * (double)first / (double)(KT_ + 1);
        const double nhi = first == KT_ ? hi : lo + (hi - lo) * (double)(first + 1) / (double)(KT_ + 1);
        lohi[0] = nlo;
        lohi[1] = nhi;
        *done = 0u;
    }
}

// rho, pi at the pattern slots of each column (Eqs. 13-14) and
// E_j = sum_i rho_ij H_ji, N_j = sum_i rho_ij S_ji (Eq. 17), from the stored
// amplitudes at the midpoint of the final bracket.  With `stage`, a column's
// amplitude block (pattern rows x nu, contiguous) is first copied into LDS
// with coalesced loads, then each thread sums its row from there.
template <typename TA>
__global__ void __launch_bounds__(128) k_rho(DevSystem S, DevJob J, const double *mu_ptr,
                                             double kT, double *rho, double *pi, double *Ecol,
                                             double *Ncol, int stage)
{
    extern __shared__ double rho_smem[];
    TA *sa = reinterpret_cast<TA *>(rho_smem);
    __shared__ double f[kMaxNu], fe[kMaxNu];
    __shared__ double red[2][2];
    const double mu = 0.5 * (mu_ptr[0] + mu_ptr[1]);
    const int o = S.o, nu = J.nu;
    for (int c = blockIdx.x; c < J.ncols; c += gridDim.x) {
        const int j = J.cols[c];
        const int A = j / o, r = j - A * o;
        const int L = J.stats[(int64_t)c * kStats];
        for (int a = threadIdx.x; a < nu; a += blockDim.x) {
            const double e = J.eps[(int64_t)c * nu + a];
            const double fa = a < L ? fermi((e - mu) / kT) : 0.0;
            f[a] = fa;
            fe[a] = a < L ? fa * e : 0.0;
        }
        __syncthreads();
        const int64_t kb0 = S.blk_ptr[A];
        const int npat = (int)(S.blk_ptr[A + 1] - kb0) * o;
        const TA *amp = reinterpret_cast<const TA *>(J.amp) + J.amp_off[c];
        if (stage) {
            for (int e = threadIdx.x; e < npat * nu; e += blockDim.x) sa[e] = amp[e];
            __syncthreads();
        }
        const TA *src = stage ? sa : amp;
        double ep = 0.0, np_ = 0.0;
        for (int t = threadIdx.x; t < npat; t += blockDim.x) {
            double sr = 0.0, sp = 0.0;
            for (int a = 0; a < L; ++a) {
                const double am = (double)src[t * nu + a];
                sr += f[a] * am;
                sp += fe[a] * am;
            }
            const int64_t slot = ((kb0 + t / o) * o + r) * o + (t % o);
            if (rho) rho[slot] = sr;
            if (pi) pi[slot] = sp;
            ep += sr * S.Hd[slot];
            np_ += sr * S.Sd[slot];
        }
        ep = wave_sum(ep);
        np_ = wave_sum(np_);
        if ((threadIdx.x & 63) == 0) {
            red[threadIdx.x >> 6][0] = ep;
            red[threadIdx.x >> 6][1] = np_;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            Ecol[c] = red[0][0] + red[1][0];
            Ncol[c] = red[0][1] + red[1][1];
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(1024) k_sum2(const double *a, const double *b, int n, double *out)
{
    __shared__ double sa[16], sb[16];
    double x = 0.0, y = 0.0;
    const int64_t chunk = (n + blockDim.x - 1) / blockDim.x;
    const int64_t e0 = threadIdx.x * chunk, e1 = min((int64_t)n, e0 + chunk);
    for (int64_t e = e0; e < e1; ++e) {
        x += a[e];
        y += b[e];
    }
    x = wave_sum(x);
    y = wave_sum(y);
    if ((threadIdx.x & 63) == 0) {
        sa[threadIdx.x >> 6] = x;
        sb[threadIdx.x >> 6] = y;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0, t = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
            s += sa[k];
            t += sb[k];
        }
        out[0] = s;
        out[1] = t;
    }
}

}  // namespace

}  // namespace ma
namespace ma {

// Host stubs of the basis-kernel families, one translation unit each
// (ma_basis_g.hip with MA_BASIS_G_O = 4, 9, 0; ma_basis_s.hip; ma_basis_m.hip).
void *basis_g_kernel_o4(int R, int prec);
void *basis_g_kernel_o9(int R, int prec);
void *basis_g_kernel_o0(int R, int prec);
void *basis_s_kernel(int o, int nt, int nucap, int prec);
void *basis_m_kernel(int o, int prec);
void *basis_a_kernel(int o, int R, int prec);   // ma_atom.hip

}  // namespace ma
