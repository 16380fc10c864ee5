// Atom basis kernel k_basis_a: the o columns j = (A, 0..o-1) of one atom in
// lockstep, so that every pass over the region operator serves all of them.
//
// The columns of an atom share their region R_A and hence H_A and S_A
// (Sec. 3, real-space projection); their Krylov spaces differ only in the
// seeds e_j and s_j (Eq. 4).  The workspace kernel streams the region
// operator once per column and product; here one workgroup runs the inner
// CGs (Sec. 2) and the delayed two-pass Gram-Schmidt recurrences (Eqs. 6-9)
// of all o columns together, and every operator product is a block SpMM over
// the o vectors of one staged set:
//
//   pass 1  H, S of the vectors finished in the previous step (-> H U, S U;
//           FP64 values only: with FP32 values the images of a finished
//           vector come from pass 2 over its pending form, see the loop)
//   pass 2  S and H of the pending vectors (FP64 values: H only while
//           block 1 runs; FP32 values: two sets when block 2 finishes two
//           vectors per step, see the loop)
//   pass 3  H of the pending chain vectors (the Euclidean chain on s_j)
//
// The staged set lives in LDS as [row][column] (o doubles per row); a thread
// takes two rows of one atom at a time, so the o x o staged entries of a
// block's column atom, read from LDS once, serve both rows (the last pair of
// an odd o holds one row).  Everything else is per column and the workspace
// kernel's arithmetic: U, S U, H U, the chain T and the working vectors of
// each column live in a per-workgroup slice of the global workspace, one
// fused dot sweep and one update sweep per step, and each column's decisions
// are taken by its leader thread (thread k for column k) and kept in LDS.
// Breakdowns and CG convergence are per column; a column that has finished
// rides along with zero vectors.
#include "ma_device.h"

namespace ma {

// doubles of one column's slice of the workspace (rounded to 256 bytes):
// U, S U, H U (nu vectors each), the chain T (q vectors), the working
// vectors P, Z, D, P2 and nine coefficient arrays of nu + 1
__host__ __device__ int64_t atom_slice_doubles(int nu, int q, int64_t ld)
{
    const int64_t d = (3 * (int64_t)nu + q + 4) * ld + 9 * (int64_t)(nu + 1);
    return (d + 31) & ~(int64_t)31;
}

// doubles of one workgroup's workspace: o column slices and five SpMM
// result sets (column-major, ld * o each)
__host__ __device__ int64_t atom_ws_doubles(int o, int nu, int q, int64_t ld)
{
    return (int64_t)o * atom_slice_doubles(nu, q, ld) + 5 * ld * o;
}

namespace {

constexpr int NTA = 256;   // threads per workgroup
constexpr int NWA = NTA / 64;
static_assert(NTA == NTG, "comb2_rows assumes rows tid + r * 256");

enum { kNone = 0, kB1 = 1, kChain = 2 };
// source of a candidate in the paired recurrence: H of the pending block-1
// vector, a finished chain vector, or the chain vector of the step
enum { kSrcNone = 0, kSrcH = 1, kSrcT = 2, kSrcZ = 3 };

// Per-column state shared by the workgroup; column k's fields are written
// only by thread k, between barriers.
struct AState {
    int live;        // a requested column whose CG succeeded and whose basis runs
    int L, nb1, kch, ping;
    int b1_live, chain_live, has_fin, has_pend;
    int kind, need_z, tail;
    int acc_u, acc_t, new_pend, new_chain;
    int iters, nres, status, start, conv, it;
    int jl, c, slot;
    double cp_scale, ctp_scale, inv_b, inv_e, f, ft, sc;
    double rho2, alpha, beta, rho;
    float rrf, alphaf, betaf;
    // paired recurrence: pending vectors (np), whether the first is a
    // block-1 vector, chain vectors used as seeds (tq), this step's
    // candidates (nc planned, nv valid; sources c3k/c4k, chain index
    // c3m/c4m), the second pending vector's acceptance, 1/beta2, its
    // coefficient g on u1, the candidates' coefficients on u1 and u2, and
    // the scale of the second pending vector's first-pass coefficients
    int np, pk1, tq, nc, nv, c3k, c3m, c4k, c4m, acc2, defer;
    double inv_b2, g, f31, f32, f41, f42, cp2_scale;
    // three-term chain: |H t|^2 of the last chain vector and of this step's
    double hn2, hn2_next, eta;
};

// Column k's vectors in the workgroup's workspace (leading dimension ld).
// CG: Z the solution (then s_j), D the residual, P the direction; the FP32
// passes keep r, p, d in U as floats.  Basis: P the pending vector
// (projected once), Z the pending chain vector, D the H image of the step's
// candidate source, P2 the second pending vector of the paired recurrence.
// After the o slices, the SpMM results of a pass, column-major (column k at
// k * ld): RH (H x), RS (S x), RH2 (H of the chain vectors, so that RH keeps
// H of the pending vectors) and RHb, RSb (H and S of the second pending
// vectors).
struct Slices {
    double *base;
    int64_t cs, ld;
    int nu, q;
    // The column offset passes through an empty asm so that the compiler
    // forms each column's addresses where they are used, instead of
    // hoisting the addresses of every column and vector to the top of the
    // kernel (which holds them in registers through every loop).
    __device__ double *U(int k) const
    {
        int64_t off = (int64_t)k * cs;
        asm volatile("" : "+v"(off));
        return base + off;
    }
    __device__ double *SU(int k) const { return U(k) + nu * ld; }
    __device__ double *K(int k) const { return SU(k) + nu * ld; }
    __device__ double *T(int k) const { return K(k) + nu * ld; }
    __device__ double *P(int k) const { return T(k) + q * ld; }
    __device__ double *Z(int k) const { return P(k) + ld; }
    __device__ double *D(int k) const { return Z(k) + ld; }
    __device__ double *P2(int k) const { return D(k) + ld; }
    __device__ double *CA(int k) const { return P2(k) + ld; }
    __device__ double *CB(int k, int which) const { return CA(k) + (1 + which) * (nu + 1); }
    __device__ double *CAT(int k) const { return CA(k) + 3 * (nu + 1); }
    __device__ double *CTB(int k, int which) const { return CA(k) + (4 + which) * (nu + 1); }
    __device__ double *CA2(int k) const { return CA(k) + 6 * (nu + 1); }
    __device__ double *CB4(int k, int which) const { return CA(k) + (7 + which) * (nu + 1); }
    __device__ float *F(int k, int v) const { return reinterpret_cast<float *>(U(k)) + v * ld; }
};

// Sink of an SpMM pass: all columns' results of row i into the column-major
// result sets (one base pointer each, so no per-column addresses stay live
// through the operator loop).
template <int O, typename TX, bool DH, bool DS>
struct ToRows {
    TX *rh, *rs;
    int64_t ld;
    __device__ __forceinline__ void operator()(int i, const TX (&h)[O], const TX (&s)[O]) const
    {
#pragma unroll
        for (int k = 0; k < O; ++k) {
            if (DH) rh[k * ld + i] = h[k];
            if (DS) rs[k * ld + i] = s[k];
        }
    }
};

// Row-triple form of the SpMM for o = 9 with FP32 operator values: a thread
// takes three rows of one atom, so each staged entry read from LDS serves
// three rows, and a region of up to 85 atoms is one task per thread (the
// row-pair form needs five tasks per atom, the last half empty).
template <int O, typename TM, typename TX, bool DH, bool DS, typename F>
__device__ __forceinline__ void spmm_set_t(const DevSystem &S, const Col &g, const TM *__restrict__ Hv,
                                           const TM *__restrict__ Sv, const TX *xs, F &&sink)
{
    constexpr int RT = 3, G = O / RT;
    static_assert(O % RT == 0, "rows split in triples");
    const int ntask = g.n_at * G;
    for (int t = threadIdx.x; t < ntask; t += NTA) {
        const int a = t / G, r0 = (t - a * G) * RT;
        TX h[RT][O], s[RT][O];
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int k = 0; k < O; ++k) h[r][k] = s[r][k] = (TX)0;
        int64_t kb0, kb1;
        if (g.lidx) {
            kb0 = g.srp[a];
            kb1 = g.srp[a + 1];
        } else {
            kb0 = g.rp[a];
            kb1 = g.rp[a + 1];
        }
        for (int64_t kb = kb0; kb < kb1; ++kb) {
            const int2 e = g.lidx ? g.sblk[kb] : S.lblk[kb];
            const int64_t base = (int64_t)e.y * (O * O) + r0 * O;
            TM hv[RT][O], sv[RT][O];
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int c = 0; c < O; ++c) {
                    if (DH) hv[r][c] = Hv[base + r * O + c];
                    if (DS) sv[r][c] = Sv[base + r * O + c];
                }
            const TX *xr = xs + (int64_t)e.x * (O * O);
#pragma unroll
            for (int c = 0; c < O; ++c) {
                TX xv[O];
#pragma unroll
                for (int k = 0; k < O; ++k) xv[k] = xr[c * O + k];
#pragma unroll
                for (int k = 0; k < O; ++k)
#pragma unroll
                    for (int r = 0; r < RT; ++r) {
                        if (DH) h[r][k] += (TX)hv[r][c] * xv[k];
                        if (DS) s[r][k] += (TX)sv[r][c] * xv[k];
                    }
            }
        }
#pragma unroll
        for (int r = 0; r < RT; ++r) sink(a * O + r0 + r, h[r], s[r]);
    }
}

// y = M x for every column of the staged set xs (LDS [row][column], O
// columns): H when DH, S when DS.  `sink(i, h, s)` receives row i's results.
// With FP32 operator values, the next block's values are loaded while the
// current block's products run (software pipelining: one block's loads in
// flight per lane); FP64 values would not leave the registers for it.
template <int O, typename TM, typename TX, bool DH, bool DS, typename F>
__device__ __forceinline__ void spmm_set(const DevSystem &S, const Col &g, const TM *__restrict__ Hv,
                                         const TM *__restrict__ Sv, const TX *xs, F &&sink)
{
    if constexpr (O == 9 && sizeof(TM) == 4) {
        spmm_set_t<O, TM, TX, DH, DS>(S, g, Hv, Sv, xs, sink);
        return;
    }
    constexpr int G = (O + 1) / 2;   // row pairs per atom
    const int ntask = g.n_at * G;
    for (int t = threadIdx.x; t < ntask; t += NTA) {
        const int a = t / G, gp = t - a * G;
        const int r0 = 2 * gp;
        const bool two = r0 + 1 < O;
        const int r1 = two ? r0 + 1 : r0;
        TX h0[O], h1[O], s0[O], s1[O];
#pragma unroll
        for (int k = 0; k < O; ++k) h0[k] = h1[k] = s0[k] = s1[k] = (TX)0;
        int64_t kb0, kb1;
        if (g.lidx) {
            kb0 = g.srp[a];
            kb1 = g.srp[a + 1];
        } else {
            kb0 = g.rp[a];
            kb1 = g.rp[a + 1];
        }
        TM hv0[O], hv1[O], sv0[O], sv1[O];
        int ex = 0;
        auto load = [&](int64_t kb, int &bx) __attribute__((always_inline)) {
            const int2 e = g.lidx ? g.sblk[kb] : S.lblk[kb];
            bx = e.x;
            const int64_t base = (int64_t)e.y * (O * O);
#pragma unroll
            for (int c = 0; c < O; ++c) {
                if (DH) {
                    hv0[c] = Hv[base + r0 * O + c];
                    hv1[c] = Hv[base + r1 * O + c];
                }
                if (DS) {
                    sv0[c] = Sv[base + r0 * O + c];
                    sv1[c] = Sv[base + r1 * O + c];
                }
            }
        };
        constexpr bool PIPE = sizeof(TM) == 4;
        if (PIPE && kb0 < kb1) load(kb0, ex);
        for (int64_t kb = kb0; kb < kb1; ++kb) {
            if (!PIPE) load(kb, ex);
            TM ch0[O], ch1[O], cs0[O], cs1[O];
#pragma unroll
            for (int c = 0; c < O; ++c) {
                ch0[c] = hv0[c];
                ch1[c] = hv1[c];
                cs0[c] = sv0[c];
                cs1[c] = sv1[c];
            }
            const int cx = ex;
            if (PIPE && kb + 1 < kb1) load(kb + 1, ex);
            const TX *xr = xs + (int64_t)cx * (O * O);
#pragma unroll
            for (int c = 0; c < O; ++c) {
                TX xv[O];
#pragma unroll
                for (int k = 0; k < O; ++k) xv[k] = xr[c * O + k];
#pragma unroll
                for (int k = 0; k < O; ++k) {
                    if (DH) {
                        h0[k] += (TX)ch0[c] * xv[k];
                        h1[k] += (TX)ch1[c] * xv[k];
                    }
                    if (DS) {
                        s0[k] += (TX)cs0[c] * xv[k];
                        s1[k] += (TX)cs1[c] * xv[k];
                    }
                }
            }
        }
        sink(a * O + r0, h0, s0);
        if (two) sink(a * O + r1, h1, s1);
    }
}

// Stage the vectors src(k) of the columns in `mask` into xs as [row][column]
// (zeros for the other columns).  The thread's rows are i = tid + rr * NTA,
// rr < R (n <= R * NTA); the loads of KB columns are issued together before
// their LDS writes, so a batch costs one memory round trip where a loop over
// the rows of one column after another waits for every load in turn.  `safe`
// is any readable vector of n entries, read in place of the columns outside
// the mask (whose src(k) need not be valid).
template <int O, int R, typename TX, typename TS, typename F>
__device__ __forceinline__ void stage_set(TX *xs, int n, unsigned mask, const TS *safe, F &&src)
{
    constexpr int KB = 3;
#pragma unroll
    for (int k0 = 0; k0 < O; k0 += KB) {
        TX v[KB][R];
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
            if (k0 + kk >= O) continue;
            const int k = k0 + kk;
            const bool on_k = (mask >> k) & 1u;
            const TS *p = on_k ? (const TS *)src(k) : safe;
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int i = threadIdx.x + rr * NTA;
                const TS x = p[i < n ? i : 0];
                v[kk][rr] = (on_k && i < n) ? (TX)x : (TX)0;
            }
        }
#pragma unroll
        for (int kk = 0; kk < KB; ++kk)
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int i = threadIdx.x + rr * NTA;
                if (k0 + kk < O && i < n) xs[i * O + k0 + kk] = v[kk][rr];
            }
    }
}

// Workgroup sums of one value per column: out[k] = sum over the workgroup
// of the thread's term(k) for the columns in `mask` (0 for the others).
template <int O, typename F>
__device__ __forceinline__ void sum_cols(unsigned mask, F &&term, double *scratch, double *out)
{
    block_reduce<NWA, 16, 1>([&](int, double (&w)[16]) __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < 16; ++k) w[k] = (k < O && ((mask >> k) & 1u)) ? term(k) : 0.0;
    }, scratch, out);
}

// One column's share of the dot sweep: V rows against x1, x2 (o1, o2) and W
// rows against y1, y2 (p1, p2), in tasks of four stored vectors.
struct DotJob {
    const double *V, *W, *x1, *x2, *y1, *y2;
    double *o1, *o2, *p1, *p2;
    int LV, LW;
    // one more vector after V (resp. W), or null: its dots with x1, x2
    // (y1, y2) go to v1, v2 (w1, w2)
    const double *Vx, *Wx;
    double *v1, *v2, *w1, *w2;
};

template <int O>
__device__ __forceinline__ void dot_sweep_cols(const DotJob *jobs, int64_t ld, int n)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int ntask = 0;
#pragma unroll
    for (int k = 0; k < O; ++k) ntask += ((jobs[k].LV + 3) >> 2) + ((jobs[k].LW + 3) >> 2);
    for (int task = w; task < ntask; task += NWA) {
        int k = 0, tl = task;
        for (; k < O - 1; ++k) {
            const int cnt = ((jobs[k].LV + 3) >> 2) + ((jobs[k].LW + 3) >> 2);
            if (tl < cnt) break;
            tl -= cnt;
        }
        const DotJob &jb = jobs[k];
        const int nv = (jb.LV + 3) >> 2;
        const bool first = tl < nv;
        const int m0 = 4 * (first ? tl : tl - nv);
        const int L = first ? jb.LV : jb.LW;
        const int nm = min(4, L - m0);
        const double *B = first ? jb.V : jb.W;
        const double *X1 = first ? jb.x1 : jb.y1;
        const double *X2 = first ? jb.x2 : jb.y2;
        const double *v0 = B + m0 * ld;
        const double *v1 = B + (m0 + (nm > 1 ? 1 : 0)) * ld;
        const double *v2 = B + (m0 + (nm > 2 ? 2 : 0)) * ld;
        const double *v3 = B + (m0 + (nm > 3 ? 3 : 0)) * ld;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        double b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
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
            const int kk = tr_index<8>(lane);
            const int m = m0 + (kk & 3);
            double *dst = (kk < 4) ? (first ? jb.o1 : jb.p1) : (first ? jb.o2 : jb.p2);
            if ((kk & 3) < nm) dst[m] = v[0];
        }
    }
}

// The same dots with whole vectors per lane: one wavefront per (column, part)
// holds x1, x2 (rows lane + 64 r, r < RR) in registers, reads the basis
// vectors VB at a time over all rows (one round trip per batch) and reduces
// each batch across the wavefront; the extra vector (Vx, Wx) is the last of
// the sequence.  Tasks: the V parts of the columns, then the W parts, so
// that the heavier V parts spread over the wavefronts.
template <int O, int RR>
__device__ __forceinline__ void dot_sweep_rows(const DotJob *jobs, int64_t ld, int n)
{
    constexpr int VB = RR <= 8 ? 4 : 2;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int task = w; task < 2 * O; task += NWA) {
        const bool first = task < O;
        const int k = first ? task : task - O;
        const DotJob &jb = jobs[k];
        const int L = first ? jb.LV : jb.LW;
        const double *Bx = first ? jb.Vx : jb.Wx;
        const int cnt = L + (Bx ? 1 : 0);
        if (cnt == 0) continue;
        const double *B = first ? jb.V : jb.W;
        const double *X1 = first ? jb.x1 : jb.y1;
        const double *X2 = first ? jb.x2 : jb.y2;
        double *D1 = first ? jb.o1 : jb.p1, *D2 = first ? jb.o2 : jb.p2;
        double *E1 = first ? jb.v1 : jb.w1, *E2 = first ? jb.v2 : jb.w2;
        double xv[RR], zv[RR];
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            const int i = lane + 64 * r;
            const bool ok = i < n;
            xv[r] = ok ? X1[ok ? i : 0] : 0.0;
            zv[r] = ok ? X2[ok ? i : 0] : 0.0;
        }
        for (int m0 = 0; m0 < cnt; m0 += VB) {
            double e[VB][RR];
#pragma unroll
            for (int j = 0; j < VB; ++j) {
                const int m = m0 + j < cnt ? m0 + j : m0;
                const double *v = m < L ? B + (int64_t)m * ld : Bx;
#pragma unroll
                for (int r = 0; r < RR; ++r) {
                    const int i = lane + 64 * r;
                    e[j][r] = v[i < n ? i : 0];   // rows past n meet zero x
                }
            }
            double acc[2 * VB];
#pragma unroll
            for (int j = 0; j < VB; ++j) {
                double a = 0.0, b = 0.0;
#pragma unroll
                for (int r = 0; r < RR; ++r) {
                    a += e[j][r] * xv[r];
                    b += e[j][r] * zv[r];
                }
                acc[j] = a;
                acc[VB + j] = b;
            }
            wave_transpose_reduce<2 * VB>(acc);
            if (tr_writer<2 * VB>(lane)) {
                const int kk = tr_index<2 * VB>(lane);
                const int m = m0 + (kk % VB);
                if (m < cnt) {
                    if (m < L) (kk < VB ? D1 : D2)[m] = acc[0];
                    else *(kk < VB ? E1 : E2) = acc[0];
                }
            }
        }
    }
}

// One column's share of the paired dot sweep: V rows against x[0..3] (the
// pending vectors P1, P2 and the candidates c3, c4; null when absent) into
// o[0..3], then the extra vectors Vx[0], Vx[1] (S P1, S P2) against the same
// four into sc[4 e + j]; W rows against y1, y2 into p1, p2, then the extra
// vectors Wx[0], Wx[1] against them into sc[8 + 4 e + j].
struct PJob {
    const double *V, *W;
    const double *x[4], *Vx[2];
    const double *y1, *y2, *Wx[2];
    double *o[4], *p1, *p2, *sc;
    int LV, LW;
};

// dot_sweep_rows with four vectors held per lane: each basis vector read
// serves the dots of two pending vectors and two candidates.
template <int O, int RR>
__device__ __forceinline__ void dot_sweep_pairs(const PJob *jobs, int64_t ld, int n)
{
    constexpr int VB = 2;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int task = w; task < 2 * O; task += NWA) {
        const bool first = task < O;
        const int k = first ? task : task - O;
        const PJob &jb = jobs[k];
        const int L = first ? jb.LV : jb.LW;
        const double *X0 = first ? jb.Vx[0] : jb.Wx[0];
        const double *X1 = first ? jb.Vx[1] : jb.Wx[1];
        const int cnt = L + (X0 ? 1 : 0) + (X1 ? 1 : 0);
        if (cnt == 0) continue;
        const double *B = first ? jb.V : jb.W;
        const double *xp[4] = {first ? jb.x[0] : jb.y1, first ? jb.x[1] : jb.y2,
                               first ? jb.x[2] : nullptr, first ? jb.x[3] : nullptr};
        double xv[4][RR];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < RR; ++r) {
                const int i = lane + 64 * r;
                xv[j][r] = (xp[j] && i < n) ? xp[j][i < n ? i : 0] : 0.0;
            }
        for (int m0 = 0; m0 < cnt; m0 += VB) {
            double e[VB][RR];
#pragma unroll
            for (int v = 0; v < VB; ++v) {
                const int m = m0 + v < cnt ? m0 + v : m0;
                const double *vec = m < L ? B + (int64_t)m * ld : (m == L ? X0 : X1);
#pragma unroll
                for (int r = 0; r < RR; ++r) {
                    const int i = lane + 64 * r;
                    e[v][r] = vec[i < n ? i : 0];   // rows past n meet zero x
                }
            }
            double acc[4 * VB];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int v = 0; v < VB; ++v) {
                    double a = 0.0;
#pragma unroll
                    for (int r = 0; r < RR; ++r) a += e[v][r] * xv[j][r];
                    acc[j * VB + v] = a;
                }
            wave_transpose_reduce<4 * VB>(acc);
            if (tr_writer<4 * VB>(lane)) {
                const int kk = tr_index<4 * VB>(lane);
                const int j = kk / VB, m = m0 + kk % VB;
                if (m < cnt && xp[j]) {
                    if (m < L) (first ? jb.o[j] : (j == 0 ? jb.p1 : jb.p2))[m] = acc[0];
                    else jb.sc[(first ? 0 : 8) + 4 * (m - L) + j] = acc[0];
                }
            }
        }
    }
}

// comb2_rows with four coefficient vectors: s_j[rr] = sum_m V[m][i] c_j[m]
// over m < cnt on the thread's rows i = tid + rr * NTA (the same batching:
// MB vectors' loads in flight, the last batch padded at coefficient zero).
template <int R, int MB = 4>
__device__ __forceinline__ void comb4_rows(const double *__restrict__ V, int64_t ld, int cnt,
                                           const double *c1, const double *c2, const double *c3,
                                           const double *c4, int n, double (&s1)[R], double (&s2)[R],
                                           double (&s3)[R], double (&s4)[R])
{
    int off[R];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
        const int i = threadIdx.x + rr * NTA;
        off[rr] = i < n ? i : 0;
        s1[rr] = s2[rr] = s3[rr] = s4[rr] = 0.0;
    }
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
            const double c = ok ? c3[mj] : 0.0, d = ok ? c4[mj] : 0.0;
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                s1[rr] += v[j][rr] * a;
                s2[rr] += v[j][rr] * b;
                s3[rr] += v[j][rr] * c;
                s4[rr] += v[j][rr] * d;
            }
        }
    }
}

struct SmemA {
    double *xs;          // staged set: nmax * O doubles (FP32 sets use it as floats)
    double *scratch;     // NWA * 64 doubles of reduction scratch
    double *red;         // 64 reduction results
    AState *st;          // O column states
    DotJob *jobs;        // O dot-sweep jobs
    PJob *pjobs;         // O paired dot-sweep jobs
    double *psc;         // 16 scalars per column of the paired dot sweep
    int *srp;            // staged region block index
    int2 *sblk;
};

__device__ __forceinline__ bool on(unsigned m, int k) { return (m >> k) & 1u; }

template <int O, int R, int PREC>
__device__ __forceinline__ void basis_atom(const DevSystem &S, const DevJob &J, const SmemA &sm, int gpos,
                           double *ws)
{
    using TM = typename std::conditional<PREC != 0, float, double>::type;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nu = J.nu, p = J.p, q = J.q;
    const int64_t ld = S.nmax;
    Slices W{ws, atom_slice_doubles(nu, q, ld), ld, nu, q};
    double *RH = ws + O * W.cs, *RS = RH + ld * O, *RH2 = RS + ld * O;
    double *RHb = RH2 + ld * O, *RSb = RHb + ld * O;
    float *RSf = reinterpret_cast<float *>(RS);
    AState *st = sm.st;
    const int p0 = J.gstart[gpos];
    const int nb = J.gstart[gpos + 1] - p0;
    const int A = J.cols[J.order[p0]] / O;
    Col g;
    {
        const int rid = S.reg_id[A];
        g.A = A;
        g.r = 0;
        g.n_at = S.reg_len[rid];
        g.n = g.n_at * O;
        g.rp = S.lrp + S.lrp_off[rid];
        g.jl = S.jloc[A] * O;
        g.lidx = false;
        g.srp = nullptr;
        g.sblk = nullptr;
    }
    if (J.lidx) stage_col_index<NTA>(S, g, sm.srp, sm.sblk);
    const int n = g.n;
    if (tid < O) {
        AState &s = st[tid];
        const bool have = tid < nb;
        s.live = have ? 1 : 0;
        s.c = have ? J.order[p0 + tid] : 0;
        s.slot = p0 + (have ? tid : 0) - J.c0;
        s.jl = g.jl + (have ? J.cols[s.c] % O : 0);
        s.iters = s.nres = s.start = s.conv = s.it = 0;
        s.status = 0;
        s.rho2 = 1.0;
    }
    __syncthreads();
    unsigned live = 0;
#pragma unroll
    for (int k = 0; k < O; ++k)
        if (st[k].live) live |= 1u << k;
    double *xsd = sm.xs;
    float *xsf = reinterpret_cast<float *>(sm.xs);

    // ---------------- inner CGs: S_A s_k = e_jk, in lockstep (Sec. 2) ----------------
    const int nout = kNbOut * O;
#pragma unroll
    for (int k = 0; k < O; ++k) {
        double *Z = W.Z(k);
        for (int i = tid; i < n; i += NTA) Z[i] = 0.0;
    }
    if (J.x0) {
        __syncthreads();
        // predicted coefficients on the orbitals of the kNbOut nearest atoms
        for (int e = tid; e < O * nout; e += NTA) {
            const int k = e / nout, f = e - k * nout;
            if (!on(live, k)) continue;
            const int kn = f / O, c2 = f - kn * O;
            const int la = S.out_loc[(int64_t)A * kNbOut + kn];
            if (la >= 0) W.Z(k)[la * O + c2] = (double)J.x0[(int64_t)st[k].c * nout + f];
        }
        if (tid < O && on(live, tid)) st[tid].start = 1;
    }
    if (J.x0full) {
        // a start on the whole region (the kept s_j of an earlier solve)
        __syncthreads();
#pragma unroll 1
        for (int k = 0; k < O; ++k)
            if (on(live, k)) {
                double *Z = W.Z(k);
                const double *x0 = J.x0full + (int64_t)st[k].c * S.nmax;
                for (int i = tid; i < n; i += NTA) Z[i] = x0[i];
            }
        if (tid < O && on(live, tid)) st[tid].start = 3;
    }
    // FP64 true residual D = e_j - S x of the columns in `mask`; |D|^2 -> red[k]
    auto true_residual = [&](unsigned mask) __attribute__((always_inline)) {
        __syncthreads();
        stage_set<O, R, double, double>(xsd, n, mask, W.Z(0), [&](int k) { return W.Z(k); });
        __syncthreads();
        spmm_set<O, double, double, false, true>(S, g, S.Hd, S.Sd, xsd,
                                                 ToRows<O, double, false, true>{RH, RS, ld});
        __syncthreads();
        sum_cols<O>(mask, [&](int k) __attribute__((always_inline)) {
            double *D = W.D(k);
            const int jk = st[k].jl;
            double a = 0.0;
            for (int i = tid; i < n; i += NTA) {
                const double r = (i == jk ? 1.0 : 0.0) - RS[k * ld + i];
                D[i] = r;
                a += r * r;
            }
            return a;
        }, sm.scratch, sm.red);
    };
    // columns whose first residual needs the operator (a given start); with a
    // zero start it is e_j itself
    __syncthreads();
    unsigned given = 0;
#pragma unroll
    for (int k = 0; k < O; ++k)
        if (on(live, k) && st[k].start != 0) given |= 1u << k;
    if (PREC == 0) {
        if (given) true_residual(given);
        if (tid < O && on(given, tid)) {
            AState &s = st[tid];
            s.rho2 = sm.red[tid];
            ++s.nres;
            if ((s.start == 1 || s.start == 3) && !(s.rho2 < 1.0)) s.start += 1;   // the judge rejects the start
        }
        __syncthreads();
#pragma unroll 1
        for (int k = 0; k < O; ++k)
            if (on(live, k) && (st[k].start == 0 || st[k].start == 2 || st[k].start == 4)) {
                double *Z = W.Z(k), *D = W.D(k);
                for (int i = tid; i < n; i += NTA) {
                    Z[i] = 0.0;
                    D[i] = i == st[k].jl ? 1.0 : 0.0;
                }
            }
        __syncthreads();
        if (tid < O && on(live, tid) && (st[tid].start == 0 || st[tid].start == 2 || st[tid].start == 4))
            st[tid].rho2 = 1.0;
        for (int restart = 0; restart <= 3; ++restart) {
            __syncthreads();
            unsigned act = 0;
#pragma unroll
            for (int k = 0; k < O; ++k)
                if (on(live, k) && st[k].status == 0 && !st[k].conv) act |= 1u << k;
            if (!act) break;
#pragma unroll 1
            for (int k = 0; k < O; ++k)
                if (on(act, k)) {
                    double *P = W.P(k);
                    const double *D = W.D(k);
                    for (int i = tid; i < n; i += NTA) P[i] = D[i];
                }
            if (tid < O) st[tid].it = 0;
            for (;;) {
                __syncthreads();
                unsigned a2 = 0;
#pragma unroll
                for (int k = 0; k < O; ++k)
                    if (on(act, k) && st[k].status == 0 && st[k].it < n &&
                        sqrt(st[k].rho2) > J.cg_tol)
                        a2 |= 1u << k;
                if (!a2) break;
                stage_set<O, R, double, double>(xsd, n, a2, W.Z(0), [&](int k) { return W.P(k); });
                __syncthreads();
                spmm_set<O, double, double, false, true>(S, g, S.Hd, S.Sd, xsd,
                                                         ToRows<O, double, false, true>{RH, RS, ld});
                __syncthreads();
                sum_cols<O>(a2, [&](int k) __attribute__((always_inline)) {
                    const double *P = W.P(k);
                    double a = 0.0;
                    for (int i = tid; i < n; i += NTA) a += P[i] * RS[k * ld + i];
                    return a;
                }, sm.scratch, sm.red);
                if (tid < O && on(a2, tid)) {
                    AState &s = st[tid];
                    const double pq = sm.red[tid];
                    if (!(pq > 0.0)) s.status = -4;
                    else s.alpha = s.rho2 / pq;
                }
                __syncthreads();
                unsigned a3 = 0;
#pragma unroll 1
                for (int k = 0; k < O; ++k)
                    if (on(a2, k) && st[k].status == 0) a3 |= 1u << k;
                sum_cols<O>(a3, [&](int k) __attribute__((always_inline)) {
                    const double al = st[k].alpha;
                    double *Z = W.Z(k), *D = W.D(k);
                    const double *P = W.P(k);
                    double a = 0.0;
                    for (int i = tid; i < n; i += NTA) {
                        Z[i] += al * P[i];
                        const double r = D[i] - al * RS[k * ld + i];
                        D[i] = r;
                        a += r * r;
                    }
                    return a;
                }, sm.scratch, sm.red);
                if (tid < O && on(a2, tid) && st[tid].status == 0) {
                    AState &s = st[tid];
                    const double rn = sm.red[tid];
                    s.beta = rn / s.rho2;
                    s.rho2 = rn;
                    ++s.iters;
                    ++s.it;
                }
                __syncthreads();
#pragma unroll 1
                for (int k = 0; k < O; ++k)
                    if (on(a2, k) && st[k].status == 0) {
                        const double be = st[k].beta;
                        double *P = W.P(k);
                        const double *D = W.D(k);
                        for (int i = tid; i < n; i += NTA) P[i] = D[i] + be * P[i];
                    }
            }
            // judge on the true residual
            __syncthreads();
            unsigned jm = 0;
#pragma unroll
            for (int k = 0; k < O; ++k)
                if (on(act, k) && st[k].status == 0) jm |= 1u << k;
            true_residual(jm);
            if (tid < O && on(jm, tid)) {
                AState &s = st[tid];
                s.rho2 = sm.red[tid];
                ++s.nres;
                if (sqrt(s.rho2) <= J.cg_tol) s.conv = 1;
            }
        }
    } else {
        // FP32 CG passes on the normalised FP64 residual, each judged and
        // refined in FP64; r, p, d, q in FP32 (F(k, 0..3))
        for (int ref = 0; ref <= J.max_refine; ++ref) {
            __syncthreads();
            unsigned jm = 0;
#pragma unroll
            for (int k = 0; k < O; ++k)
                if (on(live, k) && st[k].status == 0 && !st[k].conv) jm |= 1u << k;
            if (!jm) break;
            const unsigned ev = ref == 0 ? (jm & given) : jm;
            if (ev) true_residual(ev);
            if (tid < O && on(ev, tid)) {
                AState &s = st[tid];
                s.rho2 = sm.red[tid];
                ++s.nres;
                if (ref == 0 && (s.start == 1 || s.start == 3) && !(s.rho2 < 1.0)) s.start += 1;
            }
            __syncthreads();
#pragma unroll 1
            for (int k = 0; k < O; ++k)
                if (on(jm, k) && ref == 0 && (st[k].start == 0 || st[k].start == 2 || st[k].start == 4)) {
                    double *Z = W.Z(k), *D = W.D(k);
                    for (int i = tid; i < n; i += NTA) {
                        Z[i] = 0.0;
                        D[i] = i == st[k].jl ? 1.0 : 0.0;
                    }
                }
            __syncthreads();
            if (tid < O && on(jm, tid)) {
                AState &s = st[tid];
                if (ref == 0 && (s.start == 0 || s.start == 2 || s.start == 4)) s.rho2 = 1.0;
                if (sqrt(s.rho2) <= J.cg_tol) s.conv = 1;
                s.rho = sqrt(s.rho2);
                s.it = 0;
            }
            __syncthreads();
            unsigned pm = 0;
#pragma unroll
            for (int k = 0; k < O; ++k)
                if (on(jm, k) && !st[k].conv) pm |= 1u << k;
            if (!pm || ref == J.max_refine) break;
            sum_cols<O>(pm, [&](int k) __attribute__((always_inline)) {
                float *rf = W.F(k, 0), *pf = W.F(k, 1), *df = W.F(k, 2);
                const double *D = W.D(k);
                const double inv = 1.0 / st[k].rho;
                float acc = 0.0f;
                for (int i = tid; i < n; i += NTA) {
                    const float r = (float)(D[i] * inv);
                    rf[i] = r;
                    pf[i] = r;
                    df[i] = 0.0f;
                    acc += r * r;
                }
                return (double)acc;
            }, sm.scratch, sm.red);
            if (tid < O && on(pm, tid)) st[tid].rrf = (float)sm.red[tid];
            float thr[O];
#pragma unroll
            for (int k = 0; k < O; ++k) thr[k] = (float)fmax(J.inner_tol, 0.1 * J.cg_tol / st[k].rho);
            for (;;) {
                __syncthreads();
                unsigned a2 = 0;
#pragma unroll
                for (int k = 0; k < O; ++k)
                    if (on(pm, k) && st[k].status == 0 && st[k].it < n && sqrtf(st[k].rrf) > thr[k])
                        a2 |= 1u << k;
                if (!a2) break;
                stage_set<O, R, float, float>(xsf, n, a2, W.F(0, 1), [&](int k) { return W.F(k, 1); });
                __syncthreads();
                spmm_set<O, float, float, false, true>(S, g, S.Hf, S.Sf, xsf,
                                                       ToRows<O, float, false, true>{nullptr, RSf, ld});
                __syncthreads();
                // p^T q, three columns' loads per round trip
                block_reduce<NWA, 16, 1>([&](int, double (&w)[16]) __attribute__((always_inline)) {
#pragma unroll
                    for (int k = 0; k < 16; ++k) w[k] = 0.0;
                    constexpr int KB = 3;
#pragma unroll
                    for (int k0 = 0; k0 < O; k0 += KB) {
                        float pv[KB][R], qv[KB][R];
#pragma unroll
                        for (int kk = 0; kk < KB; ++kk) {
                            if (k0 + kk >= O) continue;
                            const int k = k0 + kk;
                            const float *pf = W.F(k, 1), *qf = RSf + k * ld;
#pragma unroll
                            for (int rr = 0; rr < R; ++rr) {
                                const int i = tid + rr * NTA, ii = i < n ? i : 0;
                                pv[kk][rr] = pf[ii];
                                qv[kk][rr] = qf[ii];
                            }
                        }
#pragma unroll
                        for (int kk = 0; kk < KB; ++kk) {
                            if (k0 + kk >= O) continue;
                            const int k = k0 + kk;
                            float acc = 0.0f;
#pragma unroll
                            for (int rr = 0; rr < R; ++rr)
                                if (tid + rr * NTA < n) acc += pv[kk][rr] * qv[kk][rr];
                            w[k] = on(a2, k) ? (double)acc : 0.0;
                        }
                    }
                }, sm.scratch, sm.red);
                if (tid < O && on(a2, tid)) {
                    AState &s = st[tid];
                    const float pq = (float)sm.red[tid];
                    if (!(pq > 0.0f)) s.status = -4;
                    else s.alphaf = s.rrf / pq;
                }
                __syncthreads();
                unsigned a3 = 0;
#pragma unroll 1
                for (int k = 0; k < O; ++k)
                    if (on(a2, k) && st[k].status == 0) a3 |= 1u << k;
                // d += alpha p, r -= alpha q, r^T r: three columns' loads per round trip
                block_reduce<NWA, 16, 1>([&](int, double (&w)[16]) __attribute__((always_inline)) {
#pragma unroll
                    for (int k = 0; k < 16; ++k) w[k] = 0.0;
                    constexpr int KB = 3;
#pragma unroll
                    for (int k0 = 0; k0 < O; k0 += KB) {
                        float dv[KB][R], pv[KB][R], rv[KB][R], qv[KB][R];
#pragma unroll
                        for (int kk = 0; kk < KB; ++kk) {
                            if (k0 + kk >= O) continue;
                            const int k = k0 + kk;
                            const float *rf = W.F(k, 0), *pf = W.F(k, 1), *df = W.F(k, 2);
                            const float *qf = RSf + k * ld;
#pragma unroll
                            for (int rr = 0; rr < R; ++rr) {
                                const int i = tid + rr * NTA, ii = i < n ? i : 0;
                                dv[kk][rr] = df[ii];
                                pv[kk][rr] = pf[ii];
                                rv[kk][rr] = rf[ii];
                                qv[kk][rr] = qf[ii];
                            }
                        }
#pragma unroll
                        for (int kk = 0; kk < KB; ++kk) {
                            if (k0 + kk >= O) continue;
                            const int k = k0 + kk;
                            if (!on(a3, k)) continue;
                            float *rf = W.F(k, 0), *df = W.F(k, 2);
                            const float al = st[k].alphaf;
                            float acc = 0.0f;
#pragma unroll
                            for (int rr = 0; rr < R; ++rr) {
                                const int i = tid + rr * NTA;
                                if (i < n) {
                                    df[i] = dv[kk][rr] + al * pv[kk][rr];
                                    const float r = rv[kk][rr] - al * qv[kk][rr];
                                    rf[i] = r;
                                    acc += r * r;
                                }
                            }
                            w[k] = (double)acc;
                        }
                    }
                }, sm.scratch, sm.red);
                if (tid < O && on(a2, tid) && st[tid].status == 0) {
                    AState &s = st[tid];
                    const float rn = (float)sm.red[tid];
                    s.betaf = rn / s.rrf;
                    s.rrf = rn;
                    ++s.iters;
                    ++s.it;
                }
                __syncthreads();
                // p = r + beta p, three columns' loads per round trip
                {
                    constexpr int KB = 3;
#pragma unroll
                    for (int k0 = 0; k0 < O; k0 += KB) {
                        float rv[KB][R], pv[KB][R];
#pragma unroll
                        for (int kk = 0; kk < KB; ++kk) {
                            if (k0 + kk >= O) continue;
                            const int k = k0 + kk;
                            const float *rf = W.F(k, 0), *pf = W.F(k, 1);
#pragma unroll
                            for (int rr = 0; rr < R; ++rr) {
                                const int i = tid + rr * NTA, ii = i < n ? i : 0;
                                rv[kk][rr] = rf[ii];
                                pv[kk][rr] = pf[ii];
                            }
                        }
#pragma unroll
                        for (int kk = 0; kk < KB; ++kk) {
                            if (k0 + kk >= O) continue;
                            const int k = k0 + kk;
                            if (!(on(a2, k) && st[k].status == 0)) continue;
                            float *pf = W.F(k, 1);
                            const float be = st[k].betaf;
#pragma unroll
                            for (int rr = 0; rr < R; ++rr) {
                                const int i = tid + rr * NTA;
                                if (i < n) pf[i] = rv[kk][rr] + be * pv[kk][rr];
                            }
                        }
                    }
                }
            }
            __syncthreads();
#pragma unroll 1
            for (int k = 0; k < O; ++k)
                if (on(pm, k) && st[k].status == 0) {
                    const float *df = W.F(k, 2);
                    double *Z = W.Z(k);
                    const double rho = st[k].rho;
                    for (int i = tid; i < n; i += NTA) Z[i] += rho * (double)df[i];
                }
        }
    }
    __syncthreads();
    if (tid < O && on(live, tid)) {
        AState &s = st[tid];
        if (s.status == 0 && !s.conv) s.status = -5;
        if (s.status != 0) s.live = 0;
    }
    if (J.sj_store) {
        // keep s_j for a later solve (MA_START_PREVIOUS)
        __syncthreads();
#pragma unroll 1
        for (int k = 0; k < O; ++k)
            if (on(live, k) && st[k].status == 0) {
                const int64_t jg = J.cols[st[k].c];
                const double *Z = W.Z(k);
                double *dst = J.sj_store + jg * S.nmax;
                for (int i = tid; i < n; i += NTA) dst[i] = Z[i];
                if (tid == 0) J.sj_have[jg] = 1;
            }
    }
    if (J.sj_near) {
        __syncthreads();
        // s_j on the orbitals of the kNbOut nearest atoms (training targets)
        for (int e = tid; e < O * nout; e += NTA) {
            const int k = e / nout, f = e - k * nout;
            if (!on(live, k)) continue;
            const int kn = f / O, c2 = f - kn * O;
            const int la = S.out_loc[(int64_t)A * kNbOut + kn];
            J.sj_near[(int64_t)st[k].c * nout + f] =
                (st[k].status == 0 && la >= 0) ? (float)W.Z(k)[la * O + c2] : 0.0f;
        }
    }
    __syncthreads();
    live = 0;
#pragma unroll
    for (int k = 0; k < O; ++k)
        if (st[k].live) live |= 1u << k;

    // ---------------- bases of K_p(H;e_j) + K_q(H;s_j), in lockstep (Eqs. 4, 6-9) ----------------
    // Paired form (FP32 operator values with FP64 sums, regions of at most
    // 1,024 rows).  The block-2 seeds come from the Euclidean chain on s_j,
    // which does not depend on the S-orthonormal basis; the chain therefore
    // advances one vector per step from the first step on, runs ahead while
    // block 1 is built, and block 2 then takes its seeds two at a time.  H is
    // symmetric, so the chain is the three-term (Lanczos) recurrence: each new
    // chain vector is orthogonalised against the two before it only, which
    // spans the same K_q(H; s_j) and needs no sweep over the chain.  A
    // step finishes up to two pending vectors (the second pass of the
    // delayed two-pass Gram-Schmidt, the second also against the first) and
    // projects up to two candidates once, so each dot sweep and each update
    // sweep over the stored basis serves two basis vectors.  The span is that
    // of Eq. 4: block 1 is the same recurrence as in the sequential form, and
    // every block-2 seed is a chain vector, taken in chain order.  The images
    // S u, H u of the finished vectors are derived from those of the pending
    // ones (u1 = (p1 - U a1) / beta1, u2 = (p2 - U a2 - g u1) / beta2) with
    // the second-pass terms in U a dropped, as in the sequential form.
    constexpr bool PAIRS = PREC == 2 && 4 * R <= 16;
    if constexpr (PAIRS) {
#pragma unroll 1
        for (int k = 0; k < O; ++k)
            if (on(live, k)) {
                double *P = W.P(k), *P2 = W.P2(k);
                for (int i = tid; i < n; i += NTA) {
                    P[i] = i == st[k].jl ? 1.0 : 0.0;   // block 1 starts at e_j
                    P2[i] = 0.0;
                }
            }
        // (the chain starts at s_j, which the CG left in Z)
        if (tid < O) {
            AState &s = st[tid];
            s.L = 0;
            s.nb1 = 0;
            s.kch = 0;
            s.tq = 0;
            s.ping = 0;
            s.chain_live = q > 0;
            s.np = p > 0 ? 1 : 0;
            s.pk1 = p > 0;
            s.defer = 0;
            s.cp_scale = s.cp2_scale = s.ctp_scale = 1.0;
            s.hn2 = s.hn2_next = 1.0;
            s.eta = 0.0;
        }
        const float *Hv = S.Hf, *Sv = S.Sf;
        auto src = [&](int k, int kind, int m) __attribute__((always_inline)) -> const double * {
            return kind == kSrcH ? RH + k * ld : kind == kSrcT ? W.T(k) + (int64_t)m * ld : W.Z(k);
        };
        for (;;) {
            __syncthreads();
            // plan of column tid: the sources of this step's candidates
            if (tid < O) {
                AState &s = st[tid];
                int nc = 0, k3 = kSrcNone, m3 = 0, k4 = kSrcNone, m4 = 0;
                if (s.live) {
                    if (s.np >= 1 && s.pk1 && s.nb1 + 1 < p) {
                        nc = 1;
                        k3 = kSrcH;
                    } else {
                        // block 2: finished chain vectors in chain order, then
                        // the chain vector this step finishes
                        for (int m = s.tq; nc < 2; ++m) {
                            const int kind = m < s.kch ? kSrcT : (m == s.kch && s.chain_live) ? kSrcZ : kSrcNone;
                            if (kind == kSrcNone) break;
                            if (nc == 0) {
                                k3 = kind;
                                m3 = m;
                            } else {
                                k4 = kind;
                                m4 = m;
                            }
                            ++nc;
                        }
                    }
                    if (s.np == 0 && nc == 0 && !s.chain_live) s.live = 0;
                }
                s.nc = nc;
                s.c3k = k3;
                s.c3m = m3;
                s.c4k = k4;
                s.c4m = m4;
            }
            __syncthreads();
            unsigned go = 0, m1 = 0, m2 = 0, ch = 0;
#pragma unroll
            for (int k = 0; k < O; ++k) {
                const AState &s = st[k];
                if (!s.live) continue;
                go |= 1u << k;
                if (s.np >= 1) m1 |= 1u << k;
                if (s.np == 2) m2 |= 1u << k;
                if (s.chain_live) ch |= 1u << k;
            }
            if (!go) break;
            // S and H of the pending vectors (RS, RH; RSb, RHb), H of the chain vectors (RH2)
            if (m1) {
                stage_set<O, R, double, double>(xsd, n, m1, W.Z(0), [&](int k) { return W.P(k); });
                __syncthreads();
                spmm_set<O, float, double, true, true>(S, g, Hv, Sv, xsd, ToRows<O, double, true, true>{RH, RS, ld});
                __syncthreads();
            }
            if (m2) {
                stage_set<O, R, double, double>(xsd, n, m2, W.Z(0), [&](int k) { return W.P2(k); });
                __syncthreads();
                spmm_set<O, float, double, true, true>(S, g, Hv, Sv, xsd,
                                                       ToRows<O, double, true, true>{RHb, RSb, ld});
                __syncthreads();
            }
            if (ch) {
                stage_set<O, R, double, double>(xsd, n, ch, W.Z(0), [&](int k) { return W.Z(k); });
                __syncthreads();
                spmm_set<O, float, double, true, false>(S, g, Hv, Sv, xsd,
                                                        ToRows<O, double, true, false>{RH2, nullptr, ld});
                __syncthreads();
            }
            if (tid < O) {
                const AState &s = st[tid];
                PJob &jb = sm.pjobs[tid];
                const bool a = s.live;
                jb.V = W.SU(tid);
                jb.LV = a && (s.np > 0 || s.nc > 0) ? s.L : 0;
                jb.x[0] = a && s.np >= 1 ? W.P(tid) : nullptr;
                jb.x[1] = a && s.np == 2 ? W.P2(tid) : nullptr;
                jb.x[2] = a && s.nc >= 1 ? src(tid, s.c3k, s.c3m) : nullptr;
                jb.x[3] = a && s.nc == 2 ? src(tid, s.c4k, s.c4m) : nullptr;
                jb.o[0] = W.CA(tid);
                jb.o[1] = W.CA2(tid);
                jb.o[2] = W.CB(tid, s.ping);
                jb.o[3] = W.CB4(tid, s.ping);
                jb.Vx[0] = a && s.np >= 1 ? RS + tid * ld : nullptr;
                jb.Vx[1] = a && s.np == 2 ? RSb + tid * ld : nullptr;
                jb.W = W.T(tid);
                jb.LW = 0;
                jb.y1 = W.Z(tid);
                jb.y2 = RH2 + tid * ld;
                jb.p1 = W.CAT(tid);
                jb.p2 = W.CTB(tid, s.ping);
                jb.Wx[0] = a && s.chain_live ? W.Z(tid) : nullptr;
                jb.Wx[1] = a && s.chain_live ? RH2 + tid * ld : nullptr;
                jb.sc = sm.psc + 16 * tid;
            }
            __syncthreads();
            // a1, a2 = (S U)^T p1, p2; b3, b4 = (S U)^T c3, c4; (S p1), (S p2)
            // against p1, p2, c3, c4; z^T z, z^T H z, (H z)^T (H z)
            dot_sweep_pairs<O, 4 * R>(sm.pjobs, ld, n);
            __syncthreads();

            // the coefficient sums of column k, one wavefront per column:
            // |a1|^2, |c1|^2, |a2|^2, |c2|^2 (c: first- plus second-pass
            // coefficients), a1.a2, a1.b3, a2.b3, a1.b4, a2.b4 -> scratch[16 k + 0..8]
#pragma unroll 1
            for (int k = wv; k < O; k += NWA) {
                const AState &s = st[k];
                if (!s.live) continue;
                const double *a1 = W.CA(k), *a2 = W.CA2(k);
                const double *b3 = W.CB(k, s.ping), *b4 = W.CB4(k, s.ping);
                const double *cp1 = W.CB(k, s.ping ^ 1), *cp2 = W.CB4(k, s.ping ^ 1);
                double v[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) v[j] = 0.0;
                for (int m = lane; m < s.L; m += 64) {
                    const double x1 = a1[m], x2 = a2[m], y3 = b3[m], y4 = b4[m];
                    const double c1 = s.cp_scale * cp1[m] + x1, c2 = s.cp2_scale * cp2[m] + x2;
                    v[0] += x1 * x1;
                    v[1] += c1 * c1;
                    v[2] += x2 * x2;
                    v[3] += c2 * c2;
                    v[4] += x1 * x2;
                    v[5] += x1 * y3;
                    v[6] += x2 * y3;
                    v[7] += x1 * y4;
                    v[8] += x2 * y4;
                }
                wave_transpose_reduce<16>(v);
                if (tr_writer<16>(lane)) sm.scratch[16 * k + tr_index<16>(lane)] = v[0];
            }
            __syncthreads();

            // decisions of column k, by thread k
            if (tid < O && st[tid].live) {
                AState &s = st[tid];
                const double *sc = sm.psc + 16 * tid, *d = sm.scratch + 16 * tid;
                // the first pending vector: beta1^2 = p1^T S p1 - |a1|^2
                bool acc1 = false;
                double ib1 = 1.0;
                if (s.np >= 1) {
                    const double bb = sc[0] - d[0], b0 = bb + d[1];
                    acc1 = bb > 0.0 && b0 > 0.0 && !(sqrt(bb) <= J.tau * sqrt(b0));
                    if (acc1) ib1 = 1.0 / sqrt(bb);
                }
                // the second: g = u1^T S p2, beta2^2 = p2^T S p2 - |a2|^2 - g^2.
                // g is a first-pass coefficient, as large as p2, so this
                // difference resolves beta2 only to about sqrt(eps) |p2|: when
                // beta2^2 falls below 1e-8 p2^T S p2, p2 is finished in the next
                // step instead, from w = p2 - U a2 - g u1, whose second pass
                // there is small (deferred)
                bool acc2 = false, defer = false;
                double ib2 = 1.0, gg = 0.0;
                if (s.np == 2) {
                    gg = acc1 ? (sc[1] - d[4]) * ib1 : 0.0;
                    const double bb = sc[5] - d[2] - gg * gg, b0 = bb + d[3] + gg * gg;
                    defer = acc1 && !(bb > 1e-8 * sc[5]);
                    acc2 = !defer && bb > 0.0 && b0 > 0.0 && !(sqrt(bb) <= J.tau * sqrt(b0));
                    if (acc2) ib2 = 1.0 / sqrt(bb);
                }
                // the candidates' coefficients on u1 and u2
                double f[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    if (c < s.nc) {
                        f[c][0] = acc1 ? (sc[2 + c] - d[5 + 2 * c]) * ib1 : 0.0;
                        f[c][1] = acc2 ? (sc[6 + c] - d[6 + 2 * c] - gg * f[c][0]) * ib2 : 0.0;
                    }
                // the chain vector z, already orthogonal to the two before it
                // (three-term recurrence, H symmetric): t = z / eta with
                // eta = |z|, checked against |H t_prev|, the norm before that
                // orthogonalisation; alpha = t^T H t; |H t|^2 for the next check
                bool acc_t = false;
                double eta = 1.0, ft = 0.0;
                if (s.chain_live) {
                    const double ee = sc[8], e0 = s.kch == 0 ? ee : s.hn2;
                    acc_t = ee > 0.0 && sqrt(ee) > J.tau * sqrt(e0);
                    if (acc_t) {
                        eta = sqrt(ee);
                        ft = sc[9] / ee;
                        s.hn2_next = sc[13] / ee;
                    }
                }
                // a block-1 candidate needs its source accepted, the chain
                // vector of the step its own acceptance
                int nv = s.nc;
                if (nv >= 1 && ((s.c3k == kSrcH && !acc1) || (s.c3k == kSrcZ && !acc_t))) nv = 0;
                if (nv == 2 && (defer || (s.c4k == kSrcZ && !acc_t))) nv = 1;   // w takes a pending slot
                s.acc_u = acc1;
                s.acc2 = acc2;
                s.defer = defer;
                s.eta = eta;
                s.inv_b = ib1;
                s.inv_b2 = ib2;
                s.g = gg;
                s.f31 = f[0][0];
                s.f32 = f[0][1];
                s.f41 = f[1][0];
                s.f42 = f[1][1];
                s.nv = nv;
                s.sc = s.c3k == kSrcH ? ib1 : 1.0;
                s.acc_t = acc_t;
                s.inv_e = 1.0 / eta;
                s.ft = ft;
                s.new_chain = s.chain_live && acc_t && s.kch + 1 < q;
            }
            __syncthreads();

            // update sweep: finish u1, u2 and t, project the candidates once
#pragma unroll 1
            for (int k = 0; k < O; ++k) {
                if (!on(go, k)) continue;
                const AState &s = st[k];
                const int L = s.L, kk = s.kch, nv = s.nv;
                const bool acc1 = s.acc_u, acc2 = s.acc2, acc_t = s.acc_t, new_chain = s.new_chain,
                           defer = s.defer;
                const double ib1 = s.inv_b, ib2 = s.inv_b2, gg = s.g, ie = s.inv_e, ft = s.ft;
                const double eta = kk > 0 ? s.eta : 0.0;
                const double f31 = s.f31, f32 = s.f32, f41 = s.f41, f42 = s.f42, sc3 = s.sc;
                double *U = W.U(k), *T = W.T(k), *P = W.P(k), *P2 = W.P2(k), *Z = W.Z(k);
                double *SUd = W.SU(k), *Kd = W.K(k);
                const double *C3 = nv >= 1 ? src(k, s.c3k, s.c3m) : Z;
                const double *C4 = nv == 2 ? src(k, s.c4k, s.c4m) : Z;
                const double *Tp = T + (int64_t)(kk > 0 ? kk - 1 : 0) * ld;   // the chain vector before t
                const double *RSk = RS + k * ld, *RHk = RH + k * ld;
                const double *RSbk = RSb + k * ld, *RHbk = RHb + k * ld, *RH2k = RH2 + k * ld;
                const int l2 = L + (acc1 ? 1 : 0);
                double s1[R], s2[R], s3[R], s4[R];
                comb4_rows<R>(U, ld, (acc1 || acc2 || nv > 0) ? L : 0, W.CA(k), W.CA2(k), W.CB(k, s.ping),
                              W.CB4(k, s.ping), n, s1, s2, s3, s4);
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    const int i = tid + rr * NTA;
                    if (i < n) {
                        const double u1 = acc1 ? (P[i] - s1[rr]) * ib1 : 0.0;
                        const double w2 = P2[i] - s2[rr] - gg * u1;   // p2 against U and u1
                        const double u2 = acc2 ? w2 * ib2 : 0.0;
                        const double c3 = C3[i], c4 = C4[i], zt = Z[i];
                        const double n1 = (c3 - s3[rr] - f31 * u1 - f32 * u2) * sc3;
                        const double n2 = c4 - s4[rr] - f41 * u1 - f42 * u2;
                        const double t = zt * ie;
                        // next chain vector: H t - alpha t - eta t_prev
                        const double tp = kk > 0 ? Tp[i] : 0.0;
                        const double nz = RH2k[i] * ie - ft * t - eta * tp;
                        const double rs1 = acc1 ? RSk[i] * ib1 : 0.0, rh1 = acc1 ? RHk[i] * ib1 : 0.0;
                        if (acc_t) T[kk * ld + i] = t;
                        if (acc1) {
                            U[L * ld + i] = u1;
                            SUd[L * ld + i] = rs1;
                            Kd[L * ld + i] = rh1;
                        }
                        if (acc2) {
                            U[l2 * ld + i] = u2;
                            SUd[l2 * ld + i] = (RSbk[i] - gg * rs1) * ib2;
                            Kd[l2 * ld + i] = (RHbk[i] - gg * rh1) * ib2;
                        }
                        // a deferred p2 goes first, as w
                        P[i] = defer ? w2 : nv >= 1 ? n1 : 0.0;
                        P2[i] = defer ? (nv >= 1 ? n1 : 0.0) : nv == 2 ? n2 : 0.0;
                        if (new_chain) Z[i] = nz;
                    }
                }
            }
            __syncthreads();
            if (tid < O && st[tid].live) {
                AState &s = st[tid];
                // first-pass coefficients of the new pending vectors on U
                // (from the dot sweep) and on u1, u2
                double *b3 = W.CB(tid, s.ping), *b4 = W.CB4(tid, s.ping);
                int l = s.L;
                if (s.defer) {
                    // pending 1 is w (p2's coefficients on U from both passes,
                    // and g on u1), pending 2 the candidate's projection
                    const double *cp2 = W.CB4(tid, s.ping ^ 1), *a2 = W.CA2(tid);
                    for (int m = 0; m < l; ++m) {
                        b4[m] = b3[m];
                        b3[m] = s.cp2_scale * cp2[m] + a2[m];
                    }
                    b3[l] = s.g;
                    b4[l] = s.f31;
                    ++l;
                } else {
                    if (s.acc_u) {
                        b3[l] = s.f31;
                        b4[l] = s.f41;
                        ++l;
                    }
                    if (s.acc2) {
                        b3[l] = s.f32;
                        b4[l] = s.f42;
                        ++l;
                    }
                }
                if (s.acc_t) s.hn2 = s.hn2_next;
                if (s.np >= 1 && s.pk1 && s.acc_u) ++s.nb1;   // a rejected block-1 vector ends block 1
                if (s.c3k == kSrcT || s.c3k == kSrcZ) s.tq += s.nv;
                if (s.chain_live) {
                    if (s.acc_t) {
                        ++s.kch;
                        s.chain_live = s.kch < q;
                    } else {
                        s.chain_live = 0;
                    }
                }
                s.L = l;
                s.cp_scale = s.defer ? 1.0 : s.sc;
                s.cp2_scale = s.defer ? s.sc : 1.0;
                s.np = s.defer ? 1 + (s.nv >= 1 ? 1 : 0) : s.nv;
                s.pk1 = !s.defer && s.nv >= 1 && s.c3k == kSrcH;
                s.ping ^= 1;
            }
        }
    } else {
    #pragma unroll 1
        for (int k = 0; k < O; ++k)
            if (on(live, k)) {
                double *P = W.P(k);
                for (int i = tid; i < n; i += NTA) P[i] = i == st[k].jl ? 1.0 : 0.0;   // block 1 starts at e_j
            }
        // (block 2 starts at s_j, which the CG left in Z)
        if (tid < O) {
            AState &s = st[tid];
            s.L = 0;
            s.nb1 = p > 0 ? 1 : 0;
            s.kch = 0;
            s.ping = 0;
            s.b1_live = 1;
            s.chain_live = q > 0;
            s.has_fin = 0;
            s.has_pend = p > 0;
            s.cp_scale = s.ctp_scale = 1.0;
        }
        const TM *Hv = PREC ? (const TM *)S.Hf : (const TM *)S.Hd;
        const TM *Sv = PREC ? (const TM *)S.Sf : (const TM *)S.Sd;
        // With FP32 operator values (FP64 sums: this kernel has no FP32-sum
        // mode) the images of a finished vector u = (p - U a) / beta are taken as
        // S p / beta and H p / beta from the pass over its pending form p: the
        // basis is orthonormal in the metric of the rounded S that every product
        // uses, so the dropped (S U) a / beta and K a / beta are second-pass
        // corrections at the FP64 rounding level, and pass 1 disappears.  With
        // FP64 values every image is applied to u itself.
        constexpr bool DERIVE = PREC == 2;
        for (;;) {
            __syncthreads();
            if (tid < O) {
                AState &s = st[tid];
                s.kind = (s.b1_live && s.nb1 < p) ? kB1 : s.chain_live ? kChain : kNone;
                s.need_z = s.kind == kChain && s.kch + 1 < q;
                s.tail = s.kind == kNone && !s.has_pend;
                if (!s.live || (!s.has_fin && !s.has_pend && s.kind == kNone)) s.live = 0;
            }
            __syncthreads();
            unsigned go = 0, fin = 0, b1 = 0, ch = 0, rest = 0;
    #pragma unroll
            for (int k = 0; k < O; ++k) {
                const AState &s = st[k];
                if (!s.live) continue;
                go |= 1u << k;
                if (s.has_fin) fin |= 1u << k;
                if (!s.tail) rest |= 1u << k;
                if (!s.tail && s.kind == kB1) b1 |= 1u << k;
                if (!s.tail && s.kind == kChain) ch |= 1u << k;
            }
            if (!go) break;

            // pass 1: H and S of the vectors finished in the previous step
            if (!DERIVE && fin) {
                stage_set<O, R, double, double>(xsd, n, fin, W.Z(0),
                                             [&](int k) { return W.U(k) + (st[k].L - 1) * ld; });
                __syncthreads();
                spmm_set<O, TM, double, true, true>(S, g, Hv, Sv, xsd,
                                                    ToRows<O, double, true, true>{RH, RS, ld});
                __syncthreads();
    #pragma unroll 1
                for (int k = 0; k < O; ++k) {
                    if (!on(fin, k)) continue;
                    const int64_t off = (int64_t)(st[k].L - 1) * ld;
                    double *SUk = W.SU(k) + off, *Kk = W.K(k) + off;
                    for (int i = tid; i < n; i += NTA) {
                        SUk[i] = RS[k * ld + i];
                        Kk[i] = RH[k * ld + i];
                    }
                }
                __syncthreads();
            }
            // columns with nothing left to project are done once their last
            // vector's images are stored
            if (tid < O && on(go, tid) && !on(rest, tid)) st[tid].has_fin = 0;
            if (!rest) continue;
            // pass 2: S and H of the pending vectors (RS, RH; FP64 values: H only
            // while block 1 runs)
            stage_set<O, R, double, double>(xsd, n, rest, W.Z(0), [&](int k) { return W.P(k); });
            __syncthreads();
            if (DERIVE || b1)
                spmm_set<O, TM, double, true, true>(S, g, Hv, Sv, xsd, ToRows<O, double, true, true>{RH, RS, ld});
            else
                spmm_set<O, TM, double, false, true>(S, g, Hv, Sv, xsd, ToRows<O, double, false, true>{RH, RS, ld});
            __syncthreads();
            // pass 3: H of the pending chain vectors into RH2 (RH keeps H of the
            // pending vectors, RS their S)
            if (ch) {
                stage_set<O, R, double, double>(xsd, n, ch, W.Z(0), [&](int k) { return W.Z(k); });
                __syncthreads();
                spmm_set<O, TM, double, true, false>(S, g, Hv, Sv, xsd,
                                                     ToRows<O, double, true, false>{RH2, nullptr, ld});
            }
            __syncthreads();
            if (tid < O) {
                // this step's dot-sweep jobs of column tid
                const AState &s = st[tid];
                const bool r = on(rest, tid);
                const int L = s.L;
                const int La = r && s.has_pend ? L : 0;
                const int Lb = r && s.kind != kNone ? L : 0;
                DotJob &jb = sm.jobs[tid];
                jb.V = W.SU(tid);
                jb.LV = La > Lb ? La : Lb;
                jb.x1 = W.P(tid);
                jb.x2 = on(ch, tid) ? W.Z(tid) : RH + tid * ld;
                jb.o1 = W.CA(tid);
                jb.o2 = W.CB(tid, s.ping);
                jb.W = W.T(tid);
                jb.LW = on(ch, tid) ? s.kch : 0;
                jb.y1 = W.Z(tid);
                jb.y2 = RH2 + tid * ld;
                jb.p1 = W.CAT(tid);
                jb.p2 = W.CTB(tid, s.ping);
                // and the scalars: pending^T S pending, (S pending)^T candidate
                // (red[2k], red[2k + 1]); chain^T chain, chain^T (H chain)
                // (red[32 + 2k], red[33 + 2k])
                jb.Vx = r ? RS + tid * ld : nullptr;
                jb.Wx = on(ch, tid) ? W.Z(tid) : nullptr;
                jb.v1 = sm.red + 2 * tid;
                jb.v2 = sm.red + 2 * tid + 1;
                jb.w1 = sm.red + 32 + 2 * tid;
                jb.w2 = sm.red + 33 + 2 * tid;
            }
            __syncthreads();
            // dots: a = (S U)^T pending, b = (S U)^T candidate; chain a_T, b_T;
            // the four scalars
            if constexpr (4 * R <= 16) {
                dot_sweep_rows<O, 4 * R>(sm.jobs, ld, n);
            } else {
                // regions of more than 1,024 rows: the scalars by a workgroup
                // reduction, then the dot sweep in tasks of four vectors
                block_reduce<NWA, 32, 2>([&](int grp, double (&v)[32]) __attribute__((always_inline)) {
    #pragma unroll
                    for (int k = 0; k < 32; ++k) v[k] = 0.0;
    #pragma unroll
                    for (int k = 0; k < O; ++k) {
                        const DotJob &jb = sm.jobs[k];
                        const double *X = grp == 0 ? jb.Vx : jb.Wx;
                        if (!X) continue;
                        const double *A1 = grp == 0 ? jb.x1 : jb.y1, *A2 = grp == 0 ? jb.x2 : jb.y2;
                        double x0 = 0.0, x1 = 0.0;
                        for (int i = tid; i < n; i += NTA) {
                            const double e = X[i];
                            x0 += e * A1[i];
                            x1 += e * A2[i];
                        }
                        v[2 * k] = x0;
                        v[2 * k + 1] = x1;
                    }
                }, sm.scratch, sm.red);   // ends with a barrier
                dot_sweep_cols<O>(sm.jobs, ld, n);
            }
            __syncthreads();

            // decisions of column k, by thread k (the workspace kernel's rule)
            if (tid < O && on(rest, tid)) {
                AState &s = st[tid];
                const double *ca = W.CA(tid);
                const double *cb = W.CB(tid, s.ping), *cp = W.CB(tid, s.ping ^ 1);
                const double *cat = W.CAT(tid);
                const double *ctb = W.CTB(tid, s.ping), *ctp = W.CTB(tid, s.ping ^ 1);
                const double nu_p = sm.red[2 * tid], e_p = sm.red[2 * tid + 1];
                const double nu_t = sm.red[32 + 2 * tid], e_t = sm.red[33 + 2 * tid];
                const int L = s.L;
                bool acc_u = false;
                double beta = 1.0, f = 0.0;
                if (s.has_pend) {
                    double asq = 0.0, tot = 0.0, ab = 0.0;
                    for (int m = 0; m < L; ++m) {
                        const double cm = s.cp_scale * cp[m] + ca[m];
                        asq += ca[m] * ca[m];
                        tot += cm * cm;
                        if (s.kind != kNone) ab += ca[m] * cb[m];
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
                if (s.kind == kChain) {
                    double asq = 0.0, tot = 0.0, ab = 0.0;
                    for (int m = 0; m < s.kch; ++m) {
                        const double cm = s.ctp_scale * ctp[m] + cat[m];
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
                s.acc_u = acc_u;
                s.acc_t = acc_t;
                s.new_pend = (s.kind == kB1 && acc_u) || (s.kind == kChain && acc_t);
                s.new_chain = s.need_z && acc_t;
                s.inv_b = 1.0 / beta;
                s.inv_e = 1.0 / eta;
                s.f = f;
                s.ft = ft;
                s.sc = s.kind == kB1 ? s.inv_b : 1.0;
            }
            __syncthreads();

            // update sweep: finish u and t, project the candidates once
    #pragma unroll 1
            for (int k = 0; k < O; ++k) {
                if (!on(rest, k)) continue;
                const AState &s = st[k];
                const int L = s.L;
                const int kk = s.kch;
                const bool acc_u = s.acc_u, acc_t = s.acc_t, new_pend = s.new_pend,
                           new_chain = s.new_chain, chain = s.kind == kChain;
                const double inv_b = s.inv_b, inv_e = s.inv_e, f = s.f, ft = s.ft, sc = s.sc;
                double *U = W.U(k), *T = W.T(k), *P = W.P(k), *Z = W.Z(k);
                double *SUd = W.SU(k), *Kd = W.K(k);
                // H image of the candidate source: H z (chain) or H of the pending vector
                const double *D = (chain ? RH2 : RH) + k * ld;
                const double *RSk = RS + k * ld, *RHk = RH + k * ld;
                double sa[R], sb[R], ta[R], tb[R];
                comb2_rows<R>(U, ld, (acc_u || new_pend) ? L : 0, W.CA(k), W.CB(k, s.ping), n, sa, sb);
                comb2_rows<R>(T, ld, acc_t ? kk : 0, W.CAT(k), W.CTB(k, s.ping), n, ta, tb);
    #pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    const int i = tid + rr * NTA;
                    if (i < n) {
                        const double up = P[i], zt = Z[i], hv = D[i];
                        const double u = (up - sa[rr]) * inv_b;
                        const double cand = chain ? zt : hv;
                        const double nl = (cand - sb[rr] - (acc_u ? f * u : 0.0)) * sc;
                        const double t = (zt - ta[rr]) * inv_e;
                        const double nz = (hv - tb[rr] - ft * t) * inv_e;
                        if (acc_t) T[kk * ld + i] = t;
                        if (acc_u) {
                            U[L * ld + i] = u;
                            if (DERIVE) {
                                SUd[L * ld + i] = RSk[i] * inv_b;
                                Kd[L * ld + i] = RHk[i] * inv_b;
                            }
                        }
                        P[i] = new_pend ? nl : 0.0;
                        if (new_chain) Z[i] = nz;
                    }
                }
            }
            __syncthreads();
            if (tid < O && on(rest, tid)) {
                AState &s = st[tid];
                if (s.acc_u) W.CB(tid, s.ping)[s.L] = s.f;   // coefficient of the new pending vector on u_L
                if (s.acc_t) W.CTB(tid, s.ping)[s.kch] = s.ft;
                if (s.kind == kB1) {
                    if (s.acc_u) ++s.nb1;
                    else s.b1_live = 0;
                }
                if (s.kind == kChain) {
                    if (s.acc_t) {
                        ++s.kch;
                        s.chain_live = s.kch < q;
                    } else {
                        s.chain_live = 0;
                    }
                }
                if (s.acc_u) ++s.L;
                s.cp_scale = s.sc;
                s.ctp_scale = s.inv_e;
                s.has_fin = DERIVE ? 0 : s.acc_u;
                s.has_pend = s.new_pend;
                s.ping ^= 1;
            }
        }
    }
    __syncthreads();   // basis writes visible to the whole workgroup

    // ---------------- Galerkin pairs (FP64 matrix cores) and basis rows ----------------
    // 16 x 16 output tiles of X = U^T H U and S~ = U^T S U per column, one
    // tile per wavefront at a time (the workspace kernel's tiling).
    unsigned done = 0;
    int ntiles = 0;
#pragma unroll
    for (int k = 0; k < O; ++k) {
        const bool ok = k < nb && st[k].status == 0;
        if (ok) done |= 1u << k;
        const int nt = ok ? (st[k].L + 15) >> 4 : 0;
        ntiles += nt * nt;
    }
    for (int task = wv; task < ntiles; task += NWA) {
        int k = 0, tl = task, pref = 0;
#pragma unroll
        for (int kk = 0; kk < O; ++kk) {
            const int nt = on(done, kk) ? (st[kk].L + 15) >> 4 : 0;
            if (nt > 0 && task >= pref) {
                k = kk;
                tl = task - pref;
            }
            pref += nt * nt;
        }
        const int Lc = st[k].L;
        const double *Uk = W.U(k), *SUk = W.SU(k), *Kk = W.K(k);
        double *mid = J.mid + (int64_t)st[k].slot * J.mid_stride;
        double *Xh = mid, *Xs = mid + (int64_t)nu * nu;
        const int nt = (Lc + 15) >> 4;
        const int mt = tl / nt, ntc = tl - mt * nt;
        const int m = mt * 16 + (lane & 15), nn = ntc * 16 + (lane & 15);
        const int kq = lane >> 4;
        const bool mok = m < Lc, nok = nn < Lc;
        const double *um = Uk + (int64_t)(mok ? m : 0) * ld;
        const double *kn = Kk + (int64_t)(nok ? nn : 0) * ld;
        const double *sn = SUk + (int64_t)(nok ? nn : 0) * ld;
        dbl4 ah = {0.0, 0.0, 0.0, 0.0}, as = {0.0, 0.0, 0.0, 0.0};
        for (int i0 = 0; i0 < n; i0 += 32) {
            double av[8], hv8[8], sv8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + 4 * u + kq;
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
            const int mr = mt * 16 + 4 * jj + kq, nc = ntc * 16 + (lane & 15);
            if (mr < Lc && nc < Lc) {
                Xh[mr * nu + nc] = ah[jj];
                Xs[mr * nu + nc] = as[jj];
            }
        }
    }
    // rows of U the outputs need: u at row j, S u at row j, u at the pattern rows
    const int64_t kb0 = S.blk_ptr[A];
    const int npat = (int)(S.blk_ptr[A + 1] - kb0) * O;
#pragma unroll 1
    for (int k = 0; k < O; ++k) {
        if (!on(done, k)) continue;
        const int L = st[k].L;
        const int jlk = st[k].jl;
        const double *U = W.U(k), *SU = W.SU(k);
        double *Up = J.mid + (int64_t)st[k].slot * J.mid_stride + 2 * (int64_t)nu * nu;
        for (int e = tid; e < (npat + 2) * L; e += NTA) {
            const int row = e / L, m = e - row * L;
            double v;
            if (row == 0) v = U[m * ld + jlk];
            else if (row == 1) v = SU[m * ld + jlk];
            else {
                const int tt = row - 2;
                v = U[m * ld + S.blk_loc[kb0 + tt / O] * O + (tt % O)];
            }
            Up[row * nu + m] = v;
        }
    }
    if (tid < O && tid < nb) {
        const AState &s = st[tid];
        write_stats(J, s.c, s.status == 0 ? s.L : 0, s.iters, s.nres, s.status, s.start);
    }
    __syncthreads();   // LDS state and the staged index are reused by the next atom
}

template <int O, int R, int PREC>
__global__ void __launch_bounds__(NTA, 2) k_basis_a(DevSystem S, DevJob J)
{
    extern __shared__ double smem[];
    __shared__ int s_idx;
    __shared__ AState sst[O];
    __shared__ DotJob sjobs[O];
    __shared__ PJob spjobs[O];
    __shared__ double spsc[O * 16];
    __shared__ double scratch[NWA * 64];
    __shared__ double red[64];
    SmemA sm;
    sm.xs = smem;
    sm.srp = reinterpret_cast<int *>(smem + (int64_t)S.nmax * O);
    sm.sblk = reinterpret_cast<int2 *>(sm.srp + ((S.max_nat + 2) & ~1));
    sm.scratch = scratch;
    sm.red = red;
    sm.st = sst;
    sm.jobs = sjobs;
    sm.pjobs = spjobs;
    sm.psc = spsc;
    double *ws = J.ws + (int64_t)blockIdx.x * J.ws_stride;
    drain_queues_raw(J, &s_idx, [&](int idx) __attribute__((always_inline)) {
        basis_atom<O, R, PREC>(S, J, sm, idx, ws);
    });
}

template <int O, int R>
void *pick_r(int prec)
{
    if (prec == 2) return (void *)k_basis_a<O, R, 2>;
    return (void *)k_basis_a<O, R, 0>;
}

template <int O>
void *pick_o(int R, int prec)
{
    switch (R) {
    case 1: return pick_r<O, 1>(prec);
    case 2: return pick_r<O, 2>(prec);
    case 3: return pick_r<O, 3>(prec);
    case 4: return pick_r<O, 4>(prec);
    case 6: return pick_r<O, 6>(prec);
    default: return pick_r<O, 8>(prec);
    }
}

}  // namespace

void *basis_a_kernel(int o, int R, int prec)
{
    return o == 9 ? pick_o<9>(R, prec) : pick_o<4>(R, prec);
}

}  // namespace ma
