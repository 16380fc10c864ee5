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
template <int O, int R, typename TM, bool DO_H, bool DO_S, bool DO_Z>
__device__ __forceinline__ void spmv_rows(const DevSystem &S, const Col &g, int o_rt,
                                          const TM *__restrict__ Hv, const TM *__restrict__ Sv,
                                          const TM *xa, const TM *xb, double (&hy)[R],
                                          double (&sy)[R], double (&zy)[R])
{
    const int o = O ? O : o_rt;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
        const int i = threadIdx.x + rr * NT;
        TM h = 0, s = 0, z = 0;
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
                        const TM xv = xa[xo + c];
                        if (DO_H) h += Hv[base + c] * xv;
                        if (DO_S) s += Sv[base + c] * xv;
                        if (DO_Z) z += Hv[base + c] * xb[xo + c];
                    }
                } else {
                    for (int c = 0; c < o; ++c) {
                        const TM xv = xa[xo + c];
                        if (DO_H) h += Hv[base + c] * xv;
                        if (DO_S) s += Sv[base + c] * xv;
                        if (DO_Z) z += Hv[base + c] * xb[xo + c];
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

// out[m] = V[m] . x for m < L (one wavefront per m; x in LDS).
__device__ __forceinline__ void multidot(const double *__restrict__ V, int64_t ld, int L,
                                         const double *x, int n, double *out)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int m = w; m < L; m += NW) {
        const double *v = V + m * ld;
        double acc = 0.0;
        for (int i = lane; i < n; i += 64) acc += v[i] * x[i];
        acc = wave_sum(acc);
        if (lane == 0) out[m] = acc;
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

template <int O, int R, bool MIXED>
__device__ void solve_column(const DevSystem &S, const DevJob &J, const Smem &sm, int c,
                             double *U, double *SU, double *K, double *T)
{
    using TM = typename std::conditional<MIXED, float, double>::type;
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
    const TM *Hv = MIXED ? (const TM *)S.Hf : (const TM *)S.Hd;
    const TM *Sv = MIXED ? (const TM *)S.Sf : (const TM *)S.Sd;
    TM *xaT = reinterpret_cast<TM *>(sm.xa);
    TM *xbT = reinterpret_cast<TM *>(sm.xb);
    double dummy[R];

    // ---------------- inner CG: S_A s = e_j ----------------
    double x[R];
    int iters = 0, nres = 0, status = 0;
    bool converged = false;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) x[rr] = 0.0;
    if (J.x0) {
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int i = tid + rr * NT;
            if (i < n) x[rr] = (double)J.x0[(int64_t)c * ld + i];
        }
    }
    if (!MIXED) {
        double r[R], p[R], q[R];
        // r = e_j - S x
        store_rows<R, double>(sm.xa, x, n);
        __syncthreads();
        spmv_rows<O, R, double, false, true, false>(S, g, o, S.Hd, S.Sd, sm.xa, sm.xb, dummy, q, dummy);
#pragma unroll
        for (int rr = 0; rr < R; ++rr) r[rr] = ((tid + rr * NT) == g.jl ? 1.0 : 0.0) - q[rr];
        double rho2 = block_sum(dot_rows<R>(r, r, n), sm.red);
        ++nres;
        for (int restart = 0; restart <= 3 && !converged && status == 0; ++restart) {
#pragma unroll
            for (int rr = 0; rr < R; ++rr) p[rr] = r[rr];
            for (int k = 0; k < n && sqrt(rho2) > J.cg_tol; ++k) {
                store_rows<R, double>(sm.xa, p, n);
                __syncthreads();
                spmv_rows<O, R, double, false, true, false>(S, g, o, S.Hd, S.Sd, sm.xa, sm.xb, dummy, q, dummy);
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
            spmv_rows<O, R, double, false, true, false>(S, g, o, S.Hd, S.Sd, sm.xa, sm.xb, dummy, q, dummy);
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
            spmv_rows<O, R, double, false, true, false>(S, g, o, S.Hd, S.Sd, sm.xa, sm.xb, dummy, q, dummy);
#pragma unroll
            for (int rr = 0; rr < R; ++rr) r64[rr] = ((tid + rr * NT) == g.jl ? 1.0 : 0.0) - q[rr];
            const double rho2 = block_sum(dot_rows<R>(r64, r64, n), sm.red);
            ++nres;
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
                    if (tid + rr * NT < n) xaT[tid + rr * NT] = (TM)pf[rr];
                __syncthreads();
                spmv_rows<O, R, TM, false, true, false>(S, g, o, Hv, Sv, xaT, xbT, dummy, qd, dummy);
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
            store_rows<R, TM>(xaT, l, n);
            if (chain) store_rows<R, TM>(xbT, t, n);
            __syncthreads();
            if (chain)
                spmv_rows<O, R, TM, true, true, true>(S, g, o, Hv, Sv, xaT, xbT, hv, w, zv);
            else
                spmv_rows<O, R, TM, true, true, false>(S, g, o, Hv, Sv, xaT, xbT, hv, w, zv);
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
        // Pairs (m <= nn) of the upper triangle, one per thread per pass; rows
        // are staged through LDS tiles of kTile rows of U, K and S U.  Both
        // u_m.k_n and u_n.k_m are formed and averaged (symmetrisation).
        const int np = L * (L + 1) / 2;
        double *Ht = sm.mat, *St = sm.mat + nu * nu, *Y = sm.mat + 2 * nu * nu;
        double *tU = sm.xa, *tK = sm.xa + L * kTile, *tS = sm.xa + 2 * L * kTile;
        for (int pbase = 0; pbase < np; pbase += NT) {
            const int e = pbase + tid;
            int pm = 0, pn = 0;
            if (e < np) {
                int rem = e;
                while (rem >= L - pm) { rem -= L - pm; ++pm; }
                pn = pm + rem;
            }
            double hu = 0.0, hl = 0.0, su = 0.0, sl = 0.0;
            for (int i0 = 0; i0 < n; i0 += kTile) {
                for (int f = tid; f < 3 * L * kTile; f += NT) {
                    const int which = f / (L * kTile);
                    const int rem = f - which * L * kTile;
                    const int m = rem / kTile, ii = rem - m * kTile;
                    const int i = i0 + ii;
                    const double *src = which == 0 ? U : (which == 1 ? K : SU);
                    tU[f] = i < n ? src[m * ld + i] : 0.0;
                }
                __syncthreads();
                if (e < np) {
#pragma unroll 4
                    for (int ii = 0; ii < kTile; ++ii) {
                        const double um = tU[pm * kTile + ii], un = tU[pn * kTile + ii];
                        hu += um * tK[pn * kTile + ii];
                        hl += un * tK[pm * kTile + ii];
                        su += um * tS[pn * kTile + ii];
                        sl += un * tS[pm * kTile + ii];
                    }
                }
                __syncthreads();
            }
            if (e < np) {
                const double h = 0.5 * (hu + hl), sv = 0.5 * (su + sl);
                Ht[pm * L + pn] = h;
                Ht[pn * L + pm] = h;
                St[pm * L + pn] = sv;
                St[pn * L + pm] = sv;
            }
        }
        if (tid == 0) s_flag = 0;
        __syncthreads();

        // ---------------- reduced generalised eigenproblem ----------------
        // Cholesky S~ = Lc Lc^T, in place in the lower triangle of St
        for (int jj = 0; jj < L; ++jj) {
            if (tid == 0) {
                double s = St[jj * L + jj];
                for (int k = 0; k < jj; ++k) s -= St[jj * L + k] * St[jj * L + k];
                if (!(s > 0.0)) { s_flag = 1; s = 1.0; }
                St[jj * L + jj] = sqrt(s);
            }
            __syncthreads();
            for (int i = jj + 1 + tid; i < L; i += NT) {
                double t2 = St[i * L + jj];
                for (int k = 0; k < jj; ++k) t2 -= St[i * L + k] * St[jj * L + k];
                St[i * L + jj] = t2 / St[jj * L + jj];
            }
            __syncthreads();
        }
        // W = Lc^-1 H~  -> Y
        for (int cc = tid; cc < L; cc += NT)
            for (int i = 0; i < L; ++i) {
                double t2 = Ht[i * L + cc];
                for (int k = 0; k < i; ++k) t2 -= St[i * L + k] * Y[k * L + cc];
                Y[i * L + cc] = t2 / St[i * L + i];
            }
        __syncthreads();
        // A = Lc^-1 W^T -> Ht
        for (int cc = tid; cc < L; cc += NT)
            for (int i = 0; i < L; ++i) {
                double t2 = Y[cc * L + i];
                for (int k = 0; k < i; ++k) t2 -= St[i * L + k] * Ht[k * L + cc];
                Ht[i * L + cc] = t2 / St[i * L + i];
            }
        __syncthreads();
        for (int e = tid; e < L * L; e += NT) {
            const int i = e / L, jj = e - i * L;
            if (i < jj) {
                const double v = 0.5 * (Ht[i * L + jj] + Ht[jj * L + i]);
                Ht[i * L + jj] = v;
                Ht[jj * L + i] = v;
            }
        }
        for (int e = tid; e < L * L; e += NT) Y[e] = (e / L == e % L) ? 1.0 : 0.0;
        __syncthreads();

        // parallel cyclic Jacobi (round-robin pairing of L2 = even(L) indices)
        {
            double *rot = sm.cf + 2 * kMaxNu;        // c, s per pair (kMaxNu/2 pairs)
            const int L2 = L + (L & 1);
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
                    if (tid < L2 / 2) {
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
                    }
                    __syncthreads();
                    // rows: A <- J^T A
                    for (int e = tid; e < (L2 / 2) * L; e += NT) {
                        const int kp = e / L, col = e - kp * L;
                        const int ia = kp == 0 ? 0 : 1 + (kp - 1 + round) % (L2 - 1);
                        const int ib = 1 + (L2 - 2 - kp + round) % (L2 - 1);
                        const int pp = min(ia, ib), qq = max(ia, ib);
                        if (qq < L) {
                            const double cs = rot[2 * kp], sn = rot[2 * kp + 1];
                            const double apk = Ht[pp * L + col], aqk = Ht[qq * L + col];
                            Ht[pp * L + col] = cs * apk - sn * aqk;
                            Ht[qq * L + col] = sn * apk + cs * aqk;
                        }
                    }
                    __syncthreads();
                    // columns: A <- A J, Y <- Y J
                    for (int e = tid; e < (L2 / 2) * L; e += NT) {
                        const int kp = e / L, row = e - kp * L;
                        const int ia = kp == 0 ? 0 : 1 + (kp - 1 + round) % (L2 - 1);
                        const int ib = 1 + (L2 - 2 - kp + round) % (L2 - 1);
                        const int pp = min(ia, ib), qq = max(ia, ib);
                        if (qq < L) {
                            const double cs = rot[2 * kp], sn = rot[2 * kp + 1];
                            const double akp = Ht[row * L + pp], akq = Ht[row * L + qq];
                            Ht[row * L + pp] = cs * akp - sn * akq;
                            Ht[row * L + qq] = sn * akp + cs * akq;
                            const double ykp = Y[row * L + pp], ykq = Y[row * L + qq];
                            Y[row * L + pp] = cs * ykp - sn * ykq;
                            Y[row * L + qq] = sn * ykp + cs * ykq;
                        }
                    }
                    __syncthreads();
                }
            }
        }
        // eigenvalues and their ascending ranks
        double *ev = sm.cf;                 // L values
        int *rank = reinterpret_cast<int *>(sm.cf + kMaxNu);
        for (int a = tid; a < L; a += NT) ev[a] = Ht[a * L + a];
        __syncthreads();
        for (int a = tid; a < L; a += NT) {
            int rk = 0;
            const double va = ev[a];
            for (int b = 0; b < L; ++b)
                if (ev[b] < va || (ev[b] == va && b < a)) ++rk;
            rank[a] = rk;
        }
        // C = Lc^-T Y -> Ht
        for (int cc = tid; cc < L; cc += NT)
            for (int i = L - 1; i >= 0; --i) {
                double t2 = Y[i * L + cc];
                for (int k = i + 1; k < L; ++k) t2 -= St[k * L + i] * Ht[k * L + cc];
                Ht[i * L + cc] = t2 / St[i * L + i];
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
        int32_t *st = J.stats + (int64_t)c * 4;
        st[0] = L;
        st[1] = iters;
        st[2] = nres;
        st[3] = status;
        if (status != 0) atomicMin(J.fail, c);
    }
    __syncthreads();
}

template <int O, int R, bool MIXED>
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
    for (;;) {
        if (threadIdx.x == 0) s_idx = atomicAdd(J.queue, 1);
        __syncthreads();
        const int idx = s_idx;
        __syncthreads();
        if (idx >= J.ncols) break;
        solve_column<O, R, MIXED>(S, J, sm, J.order[idx], U, SU, K, T);
    }
}

__global__ void k_reset(int *queue, int *fail)
{
    queue[0] = 0;
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
        if (e - c * nu < stats[c * 4]) {
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
        if (e - c * nu >= stats[c * 4]) continue;
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
        const int L = J.stats[(int64_t)c * 4];
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

template <int O, int R, bool MIXED>
hipError_t launch_solve_t(const DevSystem &S, const DevJob &J, int slots, hipStream_t st)
{
    const size_t smem = solve_smem_bytes(S.nmax, J.nu);
    auto kern = k_solve<O, R, MIXED>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(slots), dim3(NT), smem, st, S, J);
    return hipGetLastError();
}

template <int O, int R, bool MIXED>
hipError_t occupancy_t(const DevSystem &S, const DevJob &J, int *bpc)
{
    const size_t smem = solve_smem_bytes(S.nmax, J.nu);
    auto kern = k_solve<O, R, MIXED>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(bpc, kern, NT, smem);
}

#define MA_DISPATCH_R(FN, O, MIXED, ...)                                  \
    switch (R) {                                                          \
    case 1: return FN<O, 1, MIXED>(__VA_ARGS__);                          \
    case 2: return FN<O, 2, MIXED>(__VA_ARGS__);                          \
    case 3: return FN<O, 3, MIXED>(__VA_ARGS__);                          \
    case 4: return FN<O, 4, MIXED>(__VA_ARGS__);                          \
    case 6: return FN<O, 6, MIXED>(__VA_ARGS__);                          \
    default: return FN<O, 8, MIXED>(__VA_ARGS__);                         \
    }

#define MA_DISPATCH(FN, ...)                                              \
    const int R = solve_rows_per_thread(S.nmax);                          \
    if (S.o == 4) {                                                       \
        if (J.precision) { MA_DISPATCH_R(FN, 4, true, __VA_ARGS__) }     \
        else { MA_DISPATCH_R(FN, 4, false, __VA_ARGS__) }                \
    } else if (S.o == 9) {                                                \
        if (J.precision) { MA_DISPATCH_R(FN, 9, true, __VA_ARGS__) }     \
        else { MA_DISPATCH_R(FN, 9, false, __VA_ARGS__) }                \
    } else {                                                              \
        if (J.precision) { MA_DISPATCH_R(FN, 0, true, __VA_ARGS__) }     \
        else { MA_DISPATCH_R(FN, 0, false, __VA_ARGS__) }                \
    }

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
