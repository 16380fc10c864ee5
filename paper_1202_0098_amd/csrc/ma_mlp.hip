// Learned start vector for the inner CG loop: a 3-layer perceptron
//   y = W3^T silu(W2^T silu(W1^T x + b1) + b2) + b3
// mapping a column's descriptor (the 48 nearest atoms of atom(j): scaled
// distance and direction, plus the orbital type of j) to the coefficients of
// s_j = S^-1 e_j on the orbitals of the 12 atoms nearest to atom(j).
//
// Inference: one fused kernel, BF16 operands on the matrix cores
// (v_mfma_f32_16x16x16bf16_1k) with FP32 accumulation; the 64 rows of a
// workgroup stay in LDS between layers.  Training: FP32 tiled GEMMs and
// element-wise kernels (forward, MSE, backward, Adam).
#include <math.h>

#include <algorithm>

#include "ma_internal.h"

namespace ma {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short to_bf16(float x)
{
    // round to nearest even
    unsigned u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }

__device__ __forceinline__ float silu_grad(float z)
{
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// ---------------------------------------------------------------------------
// descriptors
// ---------------------------------------------------------------------------
__global__ void k_features(const int32_t *cols, int ncols, int o, const float *geo, int nf_geo,
                           int nf, float *feat)
{
    const int64_t total = (int64_t)ncols * nf;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / nf;
        const int f = (int)(e - c * nf);
        const int j = cols[c], A = j / o, r = j - A * o;
        feat[e] = f < nf_geo ? geo[(int64_t)A * nf_geo + f] : (f - nf_geo == r ? 1.0f : 0.0f);
    }
}

// ---------------------------------------------------------------------------
// fused BF16 inference
// ---------------------------------------------------------------------------
// One layer for the 16 rows of this wavefront: out[16 x n_out] =
// act(in[16 x k_pad] W + b), `in` and `out` bf16 rows in LDS (row strides in
// elements), W given transposed (n_out_pad x k_pad, bf16), one 16-column
// output tile after the other.
template <bool ACT, bool OUT_F32>
__device__ void mlp_layer(const unsigned short *in, int in_stride, int k_pad,
                          const unsigned short *__restrict__ Wt, const float *__restrict__ bias,
                          int n_out, unsigned short *out, int out_stride, float *outf,
                          int64_t outf_stride, int rows_valid)
{
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, kq = lane >> 4;
    const int ntile = (n_out + 15) >> 4;
    for (int t = 0; t < ntile; ++t) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        const int ncol = t * 16 + r16;                       // B column of this lane
        const unsigned short *wrow = Wt + (int64_t)ncol * k_pad;
        for (int k0 = 0; k0 < k_pad; k0 += 16) {
            bf16x4 a, b;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = (short)in[r16 * in_stride + k0 + 4 * kq + i];
                b[i] = (short)wrow[k0 + 4 * kq + i];
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
        // lane holds D[4*kq + jj][r16]
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int row = 4 * kq + jj, col = t * 16 + r16;
            if (col < n_out) {
                float v = acc[jj] + bias[col];
                if (ACT) v = silu(v);
                if (OUT_F32) {
                    if (row < rows_valid) outf[row * outf_stride + col] = v;
                } else {
                    out[row * out_stride + col] = to_bf16(v);
                }
            }
        }
    }
}

// 64 rows per workgroup of 256 threads (16 rows per wavefront).
__global__ void __launch_bounds__(256) k_mlp_infer(const float *X, int64_t n, int nf, int nf_pad,
                                                   int nh, int no, const unsigned short *W1t,
                                                   const float *b1, const unsigned short *W2t,
                                                   const float *b2, const unsigned short *W3t,
                                                   const float *b3, float *Y)
{
    extern __shared__ unsigned short lds[];
    const int w = threadIdx.x >> 6;
    const int stride_a = nf_pad > nh ? nf_pad : nh;
    unsigned short *bufA = lds + (int64_t)w * 16 * stride_a;            // x, then h2
    unsigned short *bufB = lds + (int64_t)4 * 16 * stride_a + w * 16 * nh;   // h1
    for (int64_t base = (int64_t)blockIdx.x * 64; base < n; base += (int64_t)gridDim.x * 64) {
        const int64_t r0 = base + w * 16;
        const int valid = (int)((n - r0) < 16 ? (n - r0) : 16);
        for (int e = threadIdx.x & 63; e < 16 * nf_pad; e += 64) {
            const int rr = e / nf_pad, f = e - rr * nf_pad;
            const float v = (rr < valid && f < nf) ? X[(r0 + rr) * nf + f] : 0.0f;
            bufA[rr * stride_a + f] = to_bf16(v);
        }
        __syncthreads();
        mlp_layer<true, false>(bufA, stride_a, nf_pad, W1t, b1, nh, bufB, nh, nullptr, 0, 16);
        __syncthreads();
        mlp_layer<true, false>(bufB, nh, nh, W2t, b2, nh, bufA, stride_a, nullptr, 0, 16);
        __syncthreads();
        if (valid > 0)
            mlp_layer<false, true>(bufA, stride_a, nh, W3t, b3, no, nullptr, 0, Y + r0 * no, no, valid);
        __syncthreads();
    }
}

// Transposed BF16 copy of an (rows x cols) FP32 matrix into (cols_pad x rows_pad).
__global__ void k_to_bf16_t(const float *W, int rows, int cols, int rows_pad, int cols_pad,
                            unsigned short *Wt)
{
    const int64_t total = (int64_t)cols_pad * rows_pad;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / rows_pad), r = (int)(e - (int64_t)c * rows_pad);
        Wt[e] = (r < rows && c < cols) ? to_bf16(W[(int64_t)r * cols + c]) : (unsigned short)0;
    }
}

// ---------------------------------------------------------------------------
// FP32 training kernels
// ---------------------------------------------------------------------------
// C[M x N] (row-major, ldc) = beta*C + A B (+ bias) with A(i,k) = A[i*sa0 + k*sa1],
// B(k,j) = B[k*sb0 + j*sb1]; rows of A optionally gathered through `gather`.
// If Z != nullptr, Z receives the pre-activation and C = silu(Z).
constexpr int TB = 64, TK = 16;
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const float *A, int64_t sa0,
                                              int64_t sa1, const int32_t *gather, const float *B,
                                              int64_t sb0, int64_t sb1, const float *bias,
                                              float beta, float *C, int64_t ldc, float *Z)
{
    __shared__ float sA[TK][TB + 1], sB[TK][TB + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i0 = blockIdx.y * TB, j0 = blockIdx.x * TB;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += TK) {
        for (int e = threadIdx.x; e < TK * TB; e += 256) {
            const int kk = e / TB, ii = e - kk * TB;
            const int i = i0 + ii, k = k0 + kk;
            float v = 0.f;
            if (i < M && k < K) {
                const int64_t ri = gather ? gather[i] : i;
                v = A[ri * sa0 + k * sa1];
            }
            sA[kk][ii] = v;
            const int j = j0 + ii;
            sB[kk][ii] = (j < N && k < K) ? B[k * sb0 + j * sb1] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = sA[kk][ty * 4 + u];
                b[u] = sB[kk][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + ty * 4 + u, j = j0 + tx * 4 + v;
            if (i < M && j < N) {
                float r = acc[u][v] + (bias ? bias[j] : 0.f);
                if (beta != 0.f) r += beta * C[i * ldc + j];
                if (Z) {
                    Z[i * ldc + j] = r;
                    r = silu(r);
                }
                C[i * ldc + j] = r;
            }
        }
}

// dY = 2 (Y - T) / (n * no); partial sums of (Y - T)^2 per block.
__global__ void __launch_bounds__(256) k_mse(const float *Y, const float *T, const int32_t *gather,
                                             int64_t n, int no, float *dY, double *partial)
{
    __shared__ double red[4];
    double s = 0.0;
    const int64_t total = n * no;
    const float scale = 2.0f / (float)total;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / no;
        const int c = (int)(e - i * no);
        const int64_t ri = gather ? gather[i] : i;
        const float d = Y[e] - T[ri * no + c];
        dY[e] = scale * d;
        s += (double)d * d;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// G = G * silu'(Z)
__global__ void k_silu_bwd(float *G, const float *Z, int64_t total)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x)
        G[e] *= silu_grad(Z[e]);
}

// db[j] = sum_i G[i, j]  (fixed order)
__global__ void k_colsum(const float *G, int64_t n, int m, float *db)
{
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int64_t i = 0; i < n; ++i) s += G[i * m + j];
        db[j] = s;
    }
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t count, float lr,
                       float b1, float b2, float eps, float c1, float c2)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        const float gg = g[e];
        const float mm = b1 * m[e] + (1.f - b1) * gg;
        const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
        m[e] = mm;
        v[e] = vv;
        p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    }
}

// out row i = in row idx[i]; an index outside [0, rows) writes zeros and
// sets *bad
__global__ void k_gather_rows(const float *in, const int32_t *idx, int64_t n, int m, int64_t rows,
                              float *out, int *bad)
{
    const int64_t total = n * m;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / m;
        const int64_t r = idx[i];
        const bool ok = r >= 0 && r < rows;
        if (!ok && e == i * m) atomicOr(bad, 1);
        out[e] = ok ? in[r * m + (e - i * m)] : 0.0f;
    }
}

inline int grid_for(int64_t n, int block) { return (int)std::min<int64_t>(4096, (n + block - 1) / block); }

}  // namespace

hipError_t launch_features(const int32_t *cols, int ncols, int o, const float *geo, int nf_geo,
                           int nf, float *feat, hipStream_t st)
{
    hipLaunchKernelGGL(k_features, dim3(grid_for((int64_t)ncols * nf, 256)), dim3(256), 0, st, cols,
                       ncols, o, geo, nf_geo, nf, feat);
    return hipGetLastError();
}

hipError_t launch_gather_rows(const float *in, const int32_t *idx, int64_t n, int m, int64_t rows,
                              float *out, int *bad, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather_rows, dim3(grid_for(n * m, 256)), dim3(256), 0, st, in, idx, n, m,
                       rows, out, bad);
    return hipGetLastError();
}

hipError_t launch_to_bf16_t(const float *W, int rows, int cols, int rows_pad, int cols_pad,
                            unsigned short *Wt, hipStream_t st)
{
    hipLaunchKernelGGL(k_to_bf16_t, dim3(grid_for((int64_t)rows_pad * cols_pad, 256)), dim3(256), 0,
                       st, W, rows, cols, rows_pad, cols_pad, Wt);
    return hipGetLastError();
}

size_t mlp_infer_smem(int nf_pad, int nh)
{
    const int stride_a = nf_pad > nh ? nf_pad : nh;
    return sizeof(unsigned short) * (size_t)(4 * 16 * stride_a + 4 * 16 * nh);
}

hipError_t launch_mlp_infer(const float *X, int64_t n, int nf, int nf_pad, int nh, int no,
                            const unsigned short *W1t, const float *b1, const unsigned short *W2t,
                            const float *b2, const unsigned short *W3t, const float *b3, float *Y,
                            hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const size_t smem = mlp_infer_smem(nf_pad, nh);
    hipError_t e = hipFuncSetAttribute((const void *)k_mlp_infer,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    const int grid = (int)std::min<int64_t>(8192, (n + 63) / 64);
    hipLaunchKernelGGL(k_mlp_infer, dim3(grid), dim3(256), smem, st, X, n, nf, nf_pad, nh, no, W1t,
                       b1, W2t, b2, W3t, b3, Y);
    return hipGetLastError();
}

hipError_t launch_gemm(int M, int N, int K, const float *A, int64_t sa0, int64_t sa1,
                       const int32_t *gather, const float *B, int64_t sb0, int64_t sb1,
                       const float *bias, float beta, float *C, int64_t ldc, float *Z, hipStream_t st)
{
    dim3 grid((N + TB - 1) / TB, (M + TB - 1) / TB);
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, M, N, K, A, sa0, sa1, gather, B, sb0, sb1,
                       bias, beta, C, ldc, Z);
    return hipGetLastError();
}

hipError_t launch_mse(const float *Y, const float *T, const int32_t *gather, int64_t n, int no,
                      float *dY, double *partial, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_mse, dim3(nblocks), dim3(256), 0, st, Y, T, gather, n, no, dY, partial);
    return hipGetLastError();
}

hipError_t launch_silu_bwd(float *G, const float *Z, int64_t total, hipStream_t st)
{
    hipLaunchKernelGGL(k_silu_bwd, dim3(grid_for(total, 256)), dim3(256), 0, st, G, Z, total);
    return hipGetLastError();
}

hipError_t launch_colsum(const float *G, int64_t n, int m, float *db, hipStream_t st)
{
    hipLaunchKernelGGL(k_colsum, dim3((m + 255) / 256), dim3(256), 0, st, G, n, m, db);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t count, float lr,
                       float b1, float b2, float eps, int step, hipStream_t st)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(count, 256)), dim3(256), 0, st, p, g, m, v, count, lr,
                       b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace ma
