// Device kernels of libmarnoldi (gfx950).
//
// k_solve: the per-column multiple Arnoldi solve (arXiv:1202.0098, Sec. 2),
// one workgroup per column, persistent over an atomic work queue.  Per
// column:
//   inner CG for s_j = S_A^-1 e_j                 (Sec. 2, inner CG loop)
//   S-orthonormal basis of K_p(H;e_j)+K_q(H;s_j)  (Eqs. 4, 6-9)
//   Galerkin pair H~ = U^T H U, S~ = U^T S U      (Sec. 2, Galerkin principle)
//   Cholesky of S~, cyclic Jacobi of L^-1 H~ L^-T (reduced eigenproblem)
//   Ritz vectors at the pattern rows of j         (Eq. 10, Eqs. 13-14)
// H_A, S_A are the principal submatrices of H, S on the region of atom(j)
// (real-space projection, Sec. 3), read through a per-region local block
// index.  Thread t owns local rows t, t+256, ...; the vector an SpMV reads is
// staged in LDS.  The basis U, S U, H U and the Krylov chain on s_j live in a
// per-workgroup slice of a global workspace.
//
// The remaining kernels weight the Ritz pairs with the Fermi function
// (Eqs. 13-14), bisect the chemical potential on the electron count and
// reduce the column energies (Eq. 17) in a fixed order.
#include <float.h>
#include <limits.h>
#include <math.h>

#include <type_traits>

#include "ma_internal.h"

namespace ma {

namespace {

constexpr int NT = kThreads;
constexpr int NW = kWaves;
constexpr int kTile = 16;          // rows per projection tile

__host__ __device__ inline int vec_doubles(int nmax, int nu)
{
    return 2 * nmax > 3 * kTile * nu ? 2 * nmax : 3 * kTile * nu;
}

// ------------------------------------------------------------------------
// reductions (xor butterflies give bitwise identical sums in every lane)
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

// Sum over the workgroup, in a fixed order.  Ends with a barrier, so the
// caller may overwrite shared buffers read before the call.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *red)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    T s = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) s += red[k];
    __syncthreads();
    return s;
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
};

// SpMV on the thread's own rows: hy = H x, sy = S x (x in LDS), zy = H xb.
// TM: stored operator values; TX: vector entries and accumulation.
template <int O, int R, typename TM, typename TX, bool DO_H, bool DO_S, bool DO_Z>
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
            const int64_t k0 = g.rp[a], k1 = g.rp[a + 1];
            for (int64_t kb = k0; kb < k1; ++kb) {
                const int2 e = S.lblk[kb];
                const int64_t base = (int64_t)e.y * (o * o) + ri * o;
                const int xo = e.x * o;
                if constexpr (O > 0) {
#pragma unroll
                    for (int c = 0; c < O; ++c) {
                        const TX xv = xa[xo + c];
                        if (DO_H) h += (TX)Hv[base + c] * xv;
                        if (DO_S) s += (TX)Sv[base + c] * xv;
                        if (DO_Z) z += (TX)Hv[base + c] * xb[xo + c];
                    }
                } else {
                    for (int c = 0; c < o; ++c) {
                        const TX xv = xa[xo + c];
                        if (DO_H) h += (TX)Hv[base + c] * xv;
                        if (DO_S) s += (TX)Sv[base + c] * xv;
                        if (DO_Z) z += (TX)Hv[base + c] * xb[xo + c];
                    }
                }
            }
        }
        hy[rr] = (double)h;
        sy[rr] = (double)s;
        zy[rr] = (double)z;
    }
}

template <int R, typename T>
__device__ __forceinline__ void store_rows(T *dst, const double (&v)[R], int n)
{
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
        const int i = threadIdx.x + rr * NT;
        if (i < n) dst[i] = (T)v[rr];
    }
}

template <int R>
__device__ __forceinline__ double dot_rows(const double (&a)[R], const double (&b)[R], int n)
{
    double s = 0.0;
#pragma unroll
    for (int rr = 0; rr < R; ++rr)
        if ((int)threadIdx.x + rr * NT < n) s += a[rr] * b[rr];
    return s;
}

// out[m] = V[m] . x for m < L (x in LDS).  Each wavefront takes four
// consecutive m at a time, keeping four independent load streams in flight.
__device__ __forceinline__ void multidot(const double *__restrict__ V, int64_t ld, int L,
                                         const double *x, int n, double *out)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int m0 = 4 * w; m0 < L; m0 += 4 * NW) {
        const int nm = min(4, L - m0);
        const double *v0 = V + m0 * ld;
        const double *v1 = V + (m0 + (nm > 1 ? 1 : 0)) * ld;
        const double *v2 = V + (m0 + (nm > 2 ? 2 : 0)) * ld;
        const double *v3 = V + (m0 + (nm > 3 ? 3 : 0)) * ld;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        for (int i = lane; i < n; i += 64) {
            const double xi = x[i];
            a0 += v0[i] * xi;
            a1 += v1[i] * xi;
            a2 += v2[i] * xi;
            a3 += v3[i] * xi;
        }
        a0 = wave_sum(a0);
        a1 = wave_sum(a1);
        a2 = wave_sum(a2);
        a3 = wave_sum(a3);
        if (lane == 0) {
            out[m0] = a0;
            if (nm > 1) out[m0 + 1] = a1;
            if (nm > 2) out[m0 + 2] = a2;
            if (nm > 3) out[m0 + 3] = a3;
        }
    }
}

// l -= sum_m V[m] c[m] on the thread's rows.
template <int R>
__device__ __forceinline__ void sub_comb(double (&l)[R], const double *__restrict__ V, int64_t ld,
                                         int L, const double *c, int n)
{
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
        const int i = threadIdx.x + rr * NT;
        if (i < n) {
            double acc = 0.0;
#pragma unroll 8
            for (int m = 0; m < L; ++m) acc += V[m * ld + i] * c[m];
            l[rr] -= acc;
        }
    }
}

// ------------------------------------------------------------------------
// the column kernel
// ------------------------------------------------------------------------
struct Smem {
    double *xa, *xb;     // nmax each: SpMV inputs / dot operands
    double *cf;          // 4 * kMaxNu: coefficients, Ritz data
    double *mat;         // 3 * nu^2: H~, S~ (then its Cholesky factor), Y (then C)
    double *red;         // NW
    float *redf;         // NW
};

// PREC 0: FP64 everywhere.  PREC 1: FP32 operator values, vectors and
// accumulation in every SpMV.  PREC 2: FP32 operator values, FP64 vectors and
// accumulation in the basis SpMVs.  PREC 1 and 2 run the CG in FP32 with an
// FP64 residual judge and refinement; Gram-Schmidt, projection and the
// eigensolve are FP64 in every mode.
template <int O, int R, int PREC>
__device__ void solve_column(const DevSystem &S, const DevJob &J, const Smem &sm, int c,
                             double *U, double *SU, double *K, double *T)
{
    using TM = typename std::conditional<PREC != 0, float, double>::type;
    using TX = typename std::conditional<PREC == 1, float, double>::type;
    const int o = O ? O : S.o;
    const int tid = threadIdx.x;
    const int64_t ld = S.nmax;
    const int nu = J.nu;
    __shared__ int s_flag;

    Col g;
    {
        const int j = J.cols[c];
        g.A = j / o;
        g.r = j - g.A * o;
        const int rid = S.reg_id[g.A];
        g.n_at = S.reg_len[rid];
        g.n = g.n_at * o;
        g.rp = S.lrp + S.lrp_off[rid];
        g.jl = S.jloc[g.A] * o + g.r;
    }
    const int n = g.n;
    const TM *Hv = PREC ? (const TM *)S.Hf : (const TM *)S.Hd;
    const TM *Sv = PREC ? (const TM *)S.Sf : (const TM *)S.Sd;
    TX *xaX = reinterpret_cast<TX *>(sm.xa);
    TX *xbX = reinterpret_cast<TX *>(sm.xb);
    float *xaF = reinterpret_cast<float *>(sm.xa);
    float *xbF = reinterpret_cast<float *>(sm.xb);
    double dummy[R];

    // ---------------- inner CG: S_A s = e_j ----------------
    double x[R];
    int iters = 0, nres = 0, status = 0, start = 0;
    bool converged = false;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) x[rr] = 0.0;
    const int nout = kNbOut * o;
    if (J.x0) {
        // predicted coefficients on the orbitals of the kNbOut nearest atoms
        for (int i = tid; i < n; i += NT) sm.xa[i] = 0.0;
        __syncthreads();
        for (int e = tid; e < nout; e += NT) {
            const int k = e / o, cc = e - k * o;
            const int la = S.out_loc[(int64_t)g.A * kNbOut + k];
            if (la >= 0) sm.xa[la * o + cc] = (double)J.x0[(int64_t)c * nout + e];
        }
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int i = tid + rr * NT;
            if (i < n) x[rr] = sm.xa[i];
        }
        start = 1;
        __syncthreads();
    }
    if (PREC == 0) {
        double r[R], p[R], q[R];
        // r = e_j - S x
        store_rows<R, double>(sm.xa, x, n);
        __syncthreads();
        spmv_rows<O, R, double, double, false, true, false>(S, g, o, S.Hd, S.Sd, sm.xa, sm.xb, dummy, q, dummy);
#pragma unroll
        for (int rr = 0; rr < R; ++rr) r[rr] = ((tid + rr * NT) == g.jl ? 1.0 : 0.0) - q[rr];
        double rho2 = block_sum(dot_rows<R>(r, r, n), sm.red);
        ++nres;
        if (start == 1 && !(rho2 < 1.0)) {
            // the residual judge rejects the predicted start: zero start
            start = 2;
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
                store_rows<R, double>(sm.xa, p, n);
                __syncthreads();
                spmv_rows<O, R, double, double, false, true, false>(S, g, o, S.Hd, S.Sd, sm.xa, sm.xb, dummy, q, dummy);
                const double pq = block_sum(dot_rows<R>(p, q, n), sm.red);
                if (!(pq > 0.0)) { status = -4; break; }
                const double alpha = rho2 / pq;
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    x[rr] += alpha * p[rr];
                    r[rr] -= alpha * q[rr];
                }
                const double rn = block_sum(dot_rows<R>(r, r, n), sm.red);
                const double beta = rn / rho2;
#pragma unroll
                for (int rr = 0; rr < R; ++rr) p[rr] = r[rr] + beta * p[rr];
                rho2 = rn;
                ++iters;
            }
            if (status) break;
            // judge on the true residual
            store_rows<R, double>(sm.xa, x, n);
            __syncthreads();
            spmv_rows<O, R, double, double, false, true, false>(S, g, o, S.Hd, S.Sd, sm.xa, sm.xb, dummy, q, dummy);
#pragma unroll
            for (int rr = 0; rr < R; ++rr) r[rr] = ((tid + rr * NT) == g.jl ? 1.0 : 0.0) - q[rr];
            rho2 = block_sum(dot_rows<R>(r, r, n), sm.red);
            ++nres;
            if (sqrt(rho2) <= J.cg_tol) converged = true;
        }
    } else {
        // FP32 CG passes with FP32 accumulation on the FP64 residual,
        // judged and refined in FP64.
        double q[R], r64[R];
        for (int ref = 0; ref <= J.max_refine && status == 0; ++ref) {
            store_rows<R, double>(sm.xa, x, n);
            __syncthreads();
            spmv_rows<O, R, double, double, false, true, false>(S, g, o, S.Hd, S.Sd, sm.xa, sm.xb, dummy, q, dummy);
#pragma unroll
            for (int rr = 0; rr < R; ++rr) r64[rr] = ((tid + rr * NT) == g.jl ? 1.0 : 0.0) - q[rr];
            double rho2 = block_sum(dot_rows<R>(r64, r64, n), sm.red);
            ++nres;
            if (ref == 0 && start == 1 && !(rho2 < 1.0)) {
                // the residual judge rejects the predicted start: zero start
                start = 2;
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
            rrf = block_sum(rrf, sm.redf);
            const float thr = (float)J.inner_tol;
            for (int k = 0; k < n && sqrtf(rrf) > thr; ++k) {
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
                    if (tid + rr * NT < n) xaF[tid + rr * NT] = pf[rr];
                __syncthreads();
                spmv_rows<O, R, float, float, false, true, false>(S, g, o, S.Hf, S.Sf, xaF, xbF, dummy, qd, dummy);
                float pq = 0.0f;
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
                    if (tid + rr * NT < n) pq += pf[rr] * (float)qd[rr];
                pq = block_sum(pq, sm.redf);
                if (!(pq > 0.0f)) { status = -4; break; }
                const float alpha = rrf / pq;
                float rn = 0.0f;
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    df[rr] += alpha * pf[rr];
                    rf[rr] -= alpha * (float)qd[rr];
                    if (tid + rr * NT < n) rn += rf[rr] * rf[rr];
                }
                rn = block_sum(rn, sm.redf);
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
    if (J.sj_near) {
        // s_j on the orbitals of the kNbOut nearest atoms (training targets)
        __syncthreads();
        store_rows<R, double>(sm.xa, x, n);
        __syncthreads();
        for (int e = tid; e < nout; e += NT) {
            const int k = e / o, cc = e - k * o;
            const int la = S.out_loc[(int64_t)g.A * kNbOut + k];
            J.sj_near[(int64_t)c * nout + e] = (status == 0 && la >= 0) ? (float)sm.xa[la * o + cc] : 0.0f;
        }
        __syncthreads();
    }

    int L = 0;
    if (status == 0) {
        // ---------------- basis of K_p(H;e_j) + K_q(H;s_j) ----------------
        double l[R], w[R], hv[R], zv[R], t[R];
        double *c1 = sm.cf, *c2 = sm.cf + kMaxNu;

        // One candidate (Eqs. 6-8): two classical Gram-Schmidt passes with
        // coefficients u_m^T S l, S-normalisation, breakdown test, and
        // acceptance u = l/beta, S u, H u.  With `chain`, also zv = H t.
        auto append = [&](bool chain) -> bool {
            for (int pass = 0; pass < 2; ++pass) {
                double *cc = pass ? c2 : c1;
                store_rows<R, double>(sm.xa, l, n);
                __syncthreads();
                multidot(SU, ld, L, sm.xa, n, cc);
                __syncthreads();
                sub_comb<R>(l, U, ld, L, cc, n);
            }
            store_rows<R, TX>(xaX, l, n);
            if (chain) store_rows<R, TX>(xbX, t, n);
            __syncthreads();
            if (chain)
                spmv_rows<O, R, TM, TX, true, true, true>(S, g, o, Hv, Sv, xaX, xbX, hv, w, zv);
            else
                spmv_rows<O, R, TM, TX, true, true, false>(S, g, o, Hv, Sv, xaX, xbX, hv, w, zv);
            const double bb = block_sum(dot_rows<R>(l, w, n), sm.red);
            double b0 = bb;
            for (int m = 0; m < L; ++m) b0 += (c1[m] + c2[m]) * (c1[m] + c2[m]);
            if (!(bb > 0.0) || !(b0 > 0.0) || sqrt(bb) <= J.tau * sqrt(b0)) return false;
            const double inv = 1.0 / sqrt(bb);
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int i = tid + rr * NT;
                if (i < n) {
                    U[L * ld + i] = l[rr] * inv;
                    SU[L * ld + i] = w[rr] * inv;
                    K[L * ld + i] = hv[rr] * inv;
                }
                l[rr] = hv[rr] * inv;   // next block-1 seed: H u_L
            }
            ++L;
            return true;
        };

        // block 1: seeds e_j, H u_1, H u_2, ...
#pragma unroll
        for (int rr = 0; rr < R; ++rr) l[rr] = (tid + rr * NT) == g.jl ? 1.0 : 0.0;
        for (int step = 0; step < J.p; ++step)
            if (!append(false)) break;

        // block 2: chain t_1 = s_j / |s_j|, t_{k+1} = H t_k orthonormalised
        if (J.q > 0) {
            const double ns = sqrt(block_sum(dot_rows<R>(x, x, n), sm.red));
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int i = tid + rr * NT;
                t[rr] = x[rr] / ns;
                if (i < n) T[i] = t[rr];
            }
            for (int k = 0; k < J.q; ++k) {
#pragma unroll
                for (int rr = 0; rr < R; ++rr) l[rr] = t[rr];
                const bool last = (k + 1 == J.q);
                append(!last);
                if (last) break;
                // Euclidean Gram-Schmidt of H t_k against t_1..t_k, twice
                const double eta0 = sqrt(block_sum(dot_rows<R>(zv, zv, n), sm.red));
                for (int pass = 0; pass < 2; ++pass) {
                    store_rows<R, double>(sm.xb, zv, n);
                    __syncthreads();
                    multidot(T, ld, k + 1, sm.xb, n, c1);
                    __syncthreads();
                    sub_comb<R>(zv, T, ld, k + 1, c1, n);
                }
                const double eta = sqrt(block_sum(dot_rows<R>(zv, zv, n), sm.red));
                if (!(eta > J.tau * eta0)) break;
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    const int i = tid + rr * NT;
                    t[rr] = zv[rr] / eta;
                    if (i < n) T[(k + 1) * ld + i] = t[rr];
                }
            }
        }
        __syncthreads();   // basis writes visible to the whole workgroup

        // ---------------- projection H~ = U^T K, S~ = U^T SU ----------------
        // Dense L x L products on the FP64 matrix cores: 16 x 16 output tiles,
        // v_mfma_f64_16x16x4f64 over the region rows, one tile per wavefront
        // at a time.  Lane l feeds A[l%16][l/16] = u_m[i] and
        // B[l/16][l%16] = k_n[i] (resp. (S u_n)[i]) and receives
        // D[4*j + l/16][l%16], j = 0..3.  Both triangles are formed, then
        // averaged.
        double *Ht = sm.mat, *St = sm.mat + nu * nu, *Y = sm.mat + 2 * nu * nu;
        {
            const int w = tid >> 6, lane = tid & 63;
            const int nt = (L + 15) >> 4;
            for (int tile = w; tile < nt * nt; tile += NW) {
                const int mt = tile / nt, ntc = tile - mt * nt;
                const int m = mt * 16 + (lane & 15), nn = ntc * 16 + (lane & 15);
                const int kk = lane >> 4;
                const bool mok = m < L, nok = nn < L;
                const double *um = U + (int64_t)(mok ? m : 0) * ld;
                const double *kn = K + (int64_t)(nok ? nn : 0) * ld;
                const double *sn = SU + (int64_t)(nok ? nn : 0) * ld;
                dbl4 ah = {0.0, 0.0, 0.0, 0.0}, as = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
                for (int i0 = 0; i0 < n; i0 += 4) {
                    const int i = i0 + kk;
                    const bool iok = i < n;
                    const double a = (mok && iok) ? um[i] : 0.0;
                    const double bh = (nok && iok) ? kn[i] : 0.0;
                    const double bs = (nok && iok) ? sn[i] : 0.0;
                    ah = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bh, ah, 0, 0, 0);
                    as = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bs, as, 0, 0, 0);
                }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int mr = mt * 16 + 4 * jj + kk, nc = ntc * 16 + (lane & 15);
                    if (mr < L && nc < L) {
                        Y[mr * L + nc] = ah[jj];          // unsymmetrised u_m . k_n
                        St[mr * L + nc] = as[jj];         // unsymmetrised u_m . S u_n
                    }
                }
            }
        }
        __syncthreads();
        for (int e = tid; e < L * L; e += NT) {
            const int i = e / L, jj = e - i * L;
            Ht[e] = 0.5 * (Y[i * L + jj] + Y[jj * L + i]);
        }
        __syncthreads();
        for (int e = tid; e < L * L; e += NT) {
            const int i = e / L, jj = e - i * L;
            if (i < jj) {
                const double v = 0.5 * (St[i * L + jj] + St[jj * L + i]);
                St[i * L + jj] = v;
                St[jj * L + i] = v;
            }
        }
        if (tid == 0) s_flag = 0;
        __syncthreads();

        // ---------------- reduced generalised eigenproblem ----------------
        // Wavefront 0 alone (L <= 64) computes the Cholesky factor S~ = Lc Lc^T
        // and the standard form A = Lc^-1 H~ Lc^-T, with wavefront-level
        // ordering of its LDS traffic instead of workgroup barriers; the
        // whole workgroup then runs the Jacobi sweeps; wavefront 0 forms
        // C = Lc^-T Y and the ranks of the eigenvalues.
        double *ev = sm.cf;                 // L values
        int *rank = reinterpret_cast<int *>(sm.cf + kMaxNu);
        if (tid < 64) {
            const int lane = tid;
            for (int jj = 0; jj < L; ++jj) {
                if (lane == 0) {
                    double sd = St[jj * L + jj];
                    for (int k = 0; k < jj; ++k) sd -= St[jj * L + k] * St[jj * L + k];
                    if (!(sd > 0.0)) { s_flag = 1; sd = 1.0; }
                    St[jj * L + jj] = sqrt(sd);
                }
                wave_sync();
                for (int i = jj + 1 + lane; i < L; i += 64) {
                    double t2 = St[i * L + jj];
                    for (int k = 0; k < jj; ++k) t2 -= St[i * L + k] * St[jj * L + k];
                    St[i * L + jj] = t2 / St[jj * L + jj];
                }
                wave_sync();
            }
            // W = Lc^-1 H~ -> Y (one column per lane)
            for (int cc = lane; cc < L; cc += 64)
                for (int i = 0; i < L; ++i) {
                    double t2 = Ht[i * L + cc];
                    for (int k = 0; k < i; ++k) t2 -= St[i * L + k] * Y[k * L + cc];
                    Y[i * L + cc] = t2 / St[i * L + i];
                }
            wave_sync();
            // A = Lc^-1 W^T -> Ht
            for (int cc = lane; cc < L; cc += 64)
                for (int i = 0; i < L; ++i) {
                    double t2 = Y[cc * L + i];
                    for (int k = 0; k < i; ++k) t2 -= St[i * L + k] * Ht[k * L + cc];
                    Ht[i * L + cc] = t2 / St[i * L + i];
                }
            wave_sync();
            for (int e = lane; e < L * L; e += 64) {
                const int i = e / L, jj = e - i * L;
                if (i < jj) {
                    const double v = 0.5 * (Ht[i * L + jj] + Ht[jj * L + i]);
                    Ht[i * L + jj] = v;
                    Ht[jj * L + i] = v;
                }
            }
            for (int e = lane; e < L * L; e += 64) Y[e] = (e / L == e % L) ? 1.0 : 0.0;
            wave_sync();

        }
        __syncthreads();

        // Cyclic Jacobi on A (all wavefronts).  Each round applies L2/2
        // disjoint rotations (circle-method pairing); A <- J^T A J is done as
        // independent 2x2 block updates (rows of pair k1 x columns of pair
        // k2), Y <- Y J as independent row pairs, so a round needs only the
        // barrier after the angles and the one after the updates.
        {
            double *rot = sm.cf + 2 * kMaxNu;                          // c, s per pair
            int *prs = reinterpret_cast<int *>(sm.cf + 3 * kMaxNu);   // p, q per pair
            const int L2 = L + (L & 1);
            const int npair = L2 / 2;
            constexpr int kMaxBlk = (kMaxNu / 2) * (kMaxNu / 2) / NT;   // 4
            constexpr int kMaxYi = kMaxNu * (kMaxNu / 2) / NT;          // 8
            int bk1[kMaxBlk], bk2[kMaxBlk], yr[kMaxYi], yk[kMaxYi];
#pragma unroll
            for (int u = 0; u < kMaxBlk; ++u) {
                const int e = tid + u * NT;
                bk1[u] = e < npair * npair ? e / npair : -1;
                bk2[u] = e < npair * npair ? e - (e / npair) * npair : -1;
            }
#pragma unroll
            for (int u = 0; u < kMaxYi; ++u) {
                const int e = tid + u * NT;
                yr[u] = e < L * npair ? e / npair : -1;
                yk[u] = e < L * npair ? e - (e / npair) * npair : -1;
            }
            double off_prev = INFINITY;
            for (int sweep = 0; sweep < 60 && L > 1; ++sweep) {
                double off = 0.0, fro = 0.0;
                for (int e = tid; e < L * L; e += NT) {
                    const double v = Ht[e] * Ht[e];
                    fro += v;
                    if (e / L != e % L) off += v;
                }
                off = block_sum(off, sm.red);
                fro = block_sum(fro, sm.red);
                if (off == 0.0 || off <= 1e-30 * fro) break;
                // no longer decreasing once at rounding level
                if (off <= 1e-24 * fro && off > 0.25 * off_prev) break;
                off_prev = off;
                for (int round = 0; round < L2 - 1; ++round) {
                    if (tid < npair) {
                        const int ia = tid == 0 ? 0 : 1 + (tid - 1 + round) % (L2 - 1);
                        const int ib = 1 + (L2 - 2 - tid + round) % (L2 - 1);
                        const int pp = min(ia, ib), qq = max(ia, ib);
                        double cs = 1.0, sn = 0.0;
                        if (qq < L) {
                            const double apq = Ht[pp * L + qq];
                            if (apq != 0.0) {
                                const double theta = (Ht[qq * L + qq] - Ht[pp * L + pp]) / (2.0 * apq);
                                double tt;
                                if (fabs(theta) > 1e150) tt = 0.5 / theta;
                                else tt = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                                cs = 1.0 / sqrt(tt * tt + 1.0);
                                sn = tt * cs;
                            }
                        }
                        rot[2 * tid] = cs;
                        rot[2 * tid + 1] = sn;
                        prs[2 * tid] = pp;
                        prs[2 * tid + 1] = qq;
                    }
                    __syncthreads();
#pragma unroll
                    for (int u = 0; u < kMaxBlk; ++u) {
                        if (bk1[u] < 0) continue;
                        const int ra = prs[2 * bk1[u]], rb = prs[2 * bk1[u] + 1];
                        const int ca = prs[2 * bk2[u]], cb = prs[2 * bk2[u] + 1];
                        const double c1 = rot[2 * bk1[u]], s1 = rot[2 * bk1[u] + 1];
                        const double c2 = rot[2 * bk2[u]], s2 = rot[2 * bk2[u] + 1];
                        const bool rbo = rb < L, cbo = cb < L;
                        const double x_ac = Ht[ra * L + ca];
                        const double x_ad = cbo ? Ht[ra * L + cb] : 0.0;
                        const double x_bc = rbo ? Ht[rb * L + ca] : 0.0;
                        const double x_bd = (rbo && cbo) ? Ht[rb * L + cb] : 0.0;
                        // rows (J^T .): a' = c1 a - s1 b, b' = s1 a + c1 b
                        const double y_ac = c1 * x_ac - s1 * x_bc, y_bc = s1 * x_ac + c1 * x_bc;
                        const double y_ad = c1 * x_ad - s1 * x_bd, y_bd = s1 * x_ad + c1 * x_bd;
                        // columns (. J): c' = c2 c - s2 d, d' = s2 c + c2 d
                        Ht[ra * L + ca] = c2 * y_ac - s2 * y_ad;
                        if (cbo) Ht[ra * L + cb] = s2 * y_ac + c2 * y_ad;
                        if (rbo) Ht[rb * L + ca] = c2 * y_bc - s2 * y_bd;
                        if (rbo && cbo) Ht[rb * L + cb] = s2 * y_bc + c2 * y_bd;
                    }
#pragma unroll
                    for (int u = 0; u < kMaxYi; ++u) {
                        if (yr[u] < 0) continue;
                        const int pp = prs[2 * yk[u]], qq = prs[2 * yk[u] + 1];
                        if (qq >= L) continue;
                        const double cs = rot[2 * yk[u]], sn = rot[2 * yk[u] + 1];
                        const int row = yr[u];
                        const double ykp = Y[row * L + pp], ykq = Y[row * L + qq];
                        Y[row * L + pp] = cs * ykp - sn * ykq;
                        Y[row * L + qq] = sn * ykp + cs * ykq;
                    }
                    __syncthreads();
                }
            }
        }
        if (tid < 64) {
            const int lane = tid;
            // eigenvalues and their ascending ranks
            for (int a = lane; a < L; a += 64) ev[a] = Ht[a * L + a];
            wave_sync();
            for (int a = lane; a < L; a += 64) {
                int rk = 0;
                const double va = ev[a];
                for (int bb = 0; bb < L; ++bb)
                    if (ev[bb] < va || (ev[bb] == va && bb < a)) ++rk;
                rank[a] = rk;
            }
            // C = Lc^-T Y -> Ht
            for (int cc = lane; cc < L; cc += 64)
                for (int i = L - 1; i >= 0; --i) {
                    double t2 = Y[i * L + cc];
                    for (int k = i + 1; k < L; ++k) t2 -= St[k * L + i] * Ht[k * L + cc];
                    Ht[i * L + cc] = t2 / St[i * L + i];
                }
        }
        __syncthreads();
        if (s_flag) status = -4;
    }

    // ---------------- outputs: Ritz values, weights, amplitudes ----------------
    double *ev = sm.cf;
    int *rank = reinterpret_cast<int *>(sm.cf + kMaxNu);
    double *vj = sm.cf + 2 * kMaxNu, *svj = sm.cf + 3 * kMaxNu;
    const double *C = sm.mat;
    if (status != 0) L = 0;
    for (int a = tid; a < L; a += NT) {
        double v1 = 0.0, v2 = 0.0;
        for (int m = 0; m < L; ++m) {
            v1 += U[m * ld + g.jl] * C[m * L + a];
            v2 += SU[m * ld + g.jl] * C[m * L + a];
        }
        vj[a] = v1;
        svj[a] = v2;
    }
    __syncthreads();
    double *eps_o = J.eps + (int64_t)c * nu, *wts_o = J.wts + (int64_t)c * nu;
    for (int a = tid; a < nu; a += NT) {
        if (a < L) {
            eps_o[rank[a]] = ev[a];
            wts_o[rank[a]] = vj[a] * svj[a];
        } else {
            eps_o[a] = NAN;
            wts_o[a] = 0.0;
        }
    }
    const int64_t kb0 = S.blk_ptr[g.A];
    const int npat = (int)(S.blk_ptr[g.A + 1] - kb0) * o;
    double *amp = J.amp + (int64_t)c * S.maxpat * nu;
    for (int e = tid; e < npat * nu; e += NT) {
        const int tt = e / nu, a = e - tt * nu;
        if (a < L) {
            const int i = S.blk_loc[kb0 + tt / o] * o + (tt % o);
            double v = 0.0;
            for (int m = 0; m < L; ++m) v += U[m * ld + i] * C[m * L + a];
            amp[tt * nu + rank[a]] = v * vj[a];
        } else {
            amp[tt * nu + a] = 0.0;
        }
    }
    if (tid == 0) {
        int32_t *st = J.stats + (int64_t)c * kStats;
        st[0] = L;
        st[1] = iters;
        st[2] = nres;
        st[3] = status;
        st[4] = start;
        st[5] = st[6] = st[7] = 0;
        if (status != 0) atomicMin(J.fail, c);
    }
    __syncthreads();
}

template <int O, int R, int PREC>
__global__ void __launch_bounds__(NT) k_solve(DevSystem S, DevJob J)
{
    extern __shared__ double smem[];
    __shared__ double red[NW];
    __shared__ float redf[NW];
    __shared__ int s_idx;
    Smem sm;
    sm.xa = smem;
    sm.xb = smem + S.nmax;
    sm.cf = smem + vec_doubles(S.nmax, J.nu);
    sm.mat = sm.cf + 4 * kMaxNu;
    sm.red = red;
    sm.redf = redf;
    const int64_t ld = S.nmax;
    double *U = J.ws + (int64_t)blockIdx.x * J.ws_stride;
    double *SU = U + J.nu * ld;
    double *K = SU + J.nu * ld;
    double *T = K + J.nu * ld;
    // Work queues: queue k serves order[qbounds[k] .. qbounds[k+1]); a
    // workgroup starts at queue blockIdx.x % nqueues and moves to the next
    // queue when one is exhausted.  Every queue is visited at most once, so
    // every workgroup leaves the loop.
    int qi = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            int idx = -1;
            for (; qi < J.nqueues; ++qi) {
                const int k = (blockIdx.x + qi) % J.nqueues;
                const int pos = J.qbounds[k] + atomicAdd(J.queue + k, 1);
                if (pos < J.qbounds[k + 1]) { idx = pos; break; }
            }
            s_idx = idx;
        }
        __syncthreads();
        const int idx = s_idx;
        __syncthreads();
        if (idx < 0) break;
        solve_column<O, R, PREC>(S, J, sm, J.order[idx], U, SU, K, T);
    }
}

__global__ void k_reset(int *queue, int *fail)
{
    for (int k = 0; k < kMaxQueues; ++k) queue[k] = 0;
    fail[0] = INT_MAX;
}

// ------------------------------------------------------------------------
// Fermi weighting and the chemical potential
// ------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_minmax(const double *eps, const int32_t *stats, int ncols,
                                                 int nu, double kT, double *lohi)
{
    __shared__ double smin[16], smax[16];
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t e = threadIdx.x; e < (int64_t)ncols * nu; e += blockDim.x) {
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
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
            lo = fmin(lo, smin[k]);
            hi = fmax(hi, smax[k]);
        }
        lo = fmin(lo, smin[0]);
        hi = fmax(hi, smax[0]);
        lohi[0] = lo - 50.0 * kT;
        lohi[1] = hi + 50.0 * kT;
    }
}

// Electron count sum_j sum_a f((eps_a - mu_t)/kT) w_a for the kBisectTrials
// trial potentials mu_t equally spaced inside (lo, hi); one partial per block.
__global__ void __launch_bounds__(256) k_count(const double *eps, const double *wts,
                                               const int32_t *stats, int ncols, int nu,
                                               double kT, const double *lohi, double *partial)
{
    constexpr int KT_ = kBisectTrials;
    __shared__ double sred[4][KT_];
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
}

// New bracket: the first trial whose count reaches the target closes it.
__global__ void k_bracket(const double *partial, int nblocks, double n_target, double *lohi)
{
    constexpr int KT_ = kBisectTrials;
    __shared__ double cnt[KT_];
    for (int t = threadIdx.x; t < KT_; t += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += partial[b * KT_ + t];
        cnt[t] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double lo = lohi[0], hi = lohi[1];
        int first = KT_;
        for (int t = 0; t < KT_; ++t)
            if (cnt[t] >= n_target) { first = t; break; }
        const double nlo = first == 0 ? lo : lo + (hi - lo) * (double)first / (double)(KT_ + 1);
        const double nhi = first == KT_ ? hi : lo + (hi - lo) * (double)(first + 1) / (double)(KT_ + 1);
        lohi[0] = nlo;
        lohi[1] = nhi;
    }
}

// rho, pi at the pattern slots of each column (Eqs. 13-14) and
// E_j = sum_i rho_ij H_ji, N_j = sum_i rho_ij S_ji (Eq. 17).
__global__ void __launch_bounds__(128) k_rho(DevSystem S, DevJob J, const double *mu_ptr, double mu_in,
                                             double kT, double *rho, double *pi, double *Ecol,
                                             double *Ncol)
{
    __shared__ double f[kMaxNu], fe[kMaxNu];
    __shared__ double red[2][2];
    const double mu = mu_ptr ? 0.5 * (mu_ptr[0] + mu_ptr[1]) : mu_in;
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
        const double *amp = J.amp + (int64_t)c * S.maxpat * nu;
        double ep = 0.0, np_ = 0.0;
        for (int t = threadIdx.x; t < npat; t += blockDim.x) {
            double sr = 0.0, sp = 0.0;
            for (int a = 0; a < L; ++a) {
                sr += f[a] * amp[t * nu + a];
                sp += fe[a] * amp[t * nu + a];
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

template <int O, int R, int PREC>
hipError_t launch_solve_t(const DevSystem &S, const DevJob &J, int slots, hipStream_t st)
{
    const size_t smem = solve_smem_bytes(S.nmax, J.nu);
    auto kern = k_solve<O, R, PREC>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(slots), dim3(NT), smem, st, S, J);
    return hipGetLastError();
}

template <int O, int R, int PREC>
hipError_t occupancy_t(const DevSystem &S, const DevJob &J, int *bpc)
{
    const size_t smem = solve_smem_bytes(S.nmax, J.nu);
    auto kern = k_solve<O, R, PREC>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(bpc, kern, NT, smem);
}

#define MA_DISPATCH_R(FN, O, PREC, ...)                                   \
    switch (R) {                                                          \
    case 1: return FN<O, 1, PREC>(__VA_ARGS__);                           \
    case 2: return FN<O, 2, PREC>(__VA_ARGS__);                           \
    case 3: return FN<O, 3, PREC>(__VA_ARGS__);                           \
    case 4: return FN<O, 4, PREC>(__VA_ARGS__);                           \
    case 6: return FN<O, 6, PREC>(__VA_ARGS__);                           \
    default: return FN<O, 8, PREC>(__VA_ARGS__);                          \
    }

#define MA_DISPATCH_P(FN, O, ...)                                         \
    if (J.precision == 1) { MA_DISPATCH_R(FN, O, 1, __VA_ARGS__) }       \
    else if (J.precision == 2) { MA_DISPATCH_R(FN, O, 2, __VA_ARGS__) }  \
    else { MA_DISPATCH_R(FN, O, 0, __VA_ARGS__) }

#define MA_DISPATCH(FN, ...)                                              \
    const int R = solve_rows_per_thread(S.nmax);                          \
    if (S.o == 4) { MA_DISPATCH_P(FN, 4, __VA_ARGS__) }                   \
    else if (S.o == 9) { MA_DISPATCH_P(FN, 9, __VA_ARGS__) }              \
    else { MA_DISPATCH_P(FN, 0, __VA_ARGS__) }

}  // namespace

int solve_rows_per_thread(int nmax)
{
    const int r = (nmax + NT - 1) / NT;
    if (r <= 4) return r < 1 ? 1 : r;
    if (r <= 6) return 6;
    return 8;
}

// LDS: vector area (the two SpMV inputs, or the projection tiles), the
// coefficient area and the three nu x nu matrices.
size_t solve_smem_bytes(int nmax, int nu)
{
    return sizeof(double) * ((size_t)vec_doubles(nmax, nu) + 4 * kMaxNu + 3 * nu * nu);
}

hipError_t launch_reset(int *queue, int *fail, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, st, queue, fail);
    return hipGetLastError();
}

hipError_t launch_solve(const DevSystem &S, const DevJob &J, int slots, hipStream_t st)
{
    MA_DISPATCH(launch_solve_t, S, J, slots, st)
}

hipError_t solve_occupancy(const DevSystem &S, const DevJob &J, int *bpc)
{
    MA_DISPATCH(occupancy_t, S, J, bpc)
}

hipError_t launch_minmax(const double *eps, const int32_t *stats, int ncols, int nu, double kT,
                         double *lohi, hipStream_t st)
{
    hipLaunchKernelGGL(k_minmax, dim3(1), dim3(1024), 0, st, eps, stats, ncols, nu, kT, lohi);
    return hipGetLastError();
}

hipError_t launch_bisect(const double *eps, const double *wts, const int32_t *stats, int ncols,
                         int nu, double kT, double n_target, double *lohi, double *partial,
                         hipStream_t st)
{
    for (int pass = 0; pass < kBisectPasses; ++pass) {
        hipLaunchKernelGGL(k_count, dim3(kCountBlocks), dim3(256), 0, st, eps, wts, stats, ncols,
                           nu, kT, lohi, partial);
        hipLaunchKernelGGL(k_bracket, dim3(1), dim3(64), 0, st, partial, kCountBlocks, n_target,
                           lohi);
    }
    return hipGetLastError();
}

hipError_t launch_rho(const DevSystem &S, const DevJob &J, const double *mu_ptr, double mu,
                      double kT, double *rho, double *pi, double *Ecol, double *Ncol,
                      hipStream_t st)
{
    const int grid = J.ncols < 65536 ? J.ncols : 65536;
    hipLaunchKernelGGL(k_rho, dim3(grid), dim3(128), 0, st, S, J, mu_ptr, mu, kT, rho, pi, Ecol,
                       Ncol);
    return hipGetLastError();
}

hipError_t launch_sum2(const double *a, const double *b, int n, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum2, dim3(1), dim3(1024), 0, st, a, b, n, out);
    return hipGetLastError();
}

}  // namespace ma
