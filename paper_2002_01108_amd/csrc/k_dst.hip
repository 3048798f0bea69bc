// Step 2 of the BEC inverse for a constant coefficient (Section 4,
// eq. (blockdiaginv)): each block B_k = lambda_k I + tau K_h is diagonalised
// by the orthogonal, symmetric DST-I matrix S (one per axis),
//   ztilde_k = (S x S x S) diag(1 / (lambda_k + tau mu)) (S x S x S) ytilde_k,
// the fast sine transform of the paper replaced by dense products with S on
// the matrix cores.  A mode product along one axis of the split-plane
// spectrum is a batched real GEMM (S real, planes real):
//   along x:  Out[rows][P1]     = In[rows][P1] * S          ("right")
//   along y/z: Out[b][P][R]     = S * In[b][P][R]           ("left")
// Padding rows/columns of S are zero, so zero padding in the planes stays zero.
#include "common.h"

namespace aao {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Acc;
// Accumulator layouts of the 16x16x4 MFMAs (lane l, element v; lk = l/16):
//   FP64: row lk + 4 v,  col l % 16
//   FP32: row 4 lk + v,  col l % 16
// (both measured on gfx950 against a reference product)
template <> struct Acc<double> {
  typedef d4 type;
  static __device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <> struct Acc<float> {
  typedef f4 type;
  static __device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};

constexpr int BM = 64, BN = 64, BK = 16, PADK = 1;
constexpr int GTHREADS = 256;

// C[b] = A[b] * B[b]; A M x K (lda), B K x N (ldb), C M x N (ldc), row-major.
// N, K multiples of 64 / 16; M may be ragged (rows >= M read as zero, not stored).
// 4 waves, each a 32 x 32 sub-tile of 2 x 2 MFMA 16x16x4 tiles.  LDS double
// buffer; the next K slice is fetched into registers while the current one
// feeds the matrix cores.
template <typename T>
__global__ __launch_bounds__(GTHREADS) void k_gemm(const T* __restrict__ A, int64_t sA, int lda,
                                                    const T* __restrict__ B, int64_t sB, int ldb,
                                                    T* __restrict__ C, int64_t sC, int ldc, int M,
                                                    int N, int K, int tiles_m, int tiles_n) {
  using V4 = typename Acc<T>::type;
  __shared__ T As[2][BK][BM + PADK];
  __shared__ T Bs[2][BK][BN + PADK];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  int bid = blockIdx.x;
  const int tn = bid % tiles_n;
  bid /= tiles_n;
  const int tm = bid % tiles_m;
  const int batch = bid / tiles_m;
  const int m0 = tm * BM, n0 = tn * BN;
  A += batch * sA;
  B += batch * sB;
  C += batch * sC;

  // global load assignment
  const int ar = tid >> 2, ak = (tid & 3) * 4;     // A: row ar, k ak..ak+3
  const int bk = tid >> 4, bn = (tid & 15) * 4;    // B: k bk, cols bn..bn+3
  const bool arow_ok = (m0 + ar) < M;
  const T* Ap = A + (int64_t)(arow_ok ? m0 + ar : 0) * lda + ak;
  const T* Bp = B + (int64_t)bk * ldb + n0 + bn;

  T ra[4], rb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) ra[e] = arow_ok ? Ap[k0 + e] : T(0);
#pragma unroll
    for (int e = 0; e < 4; ++e) rb[e] = Bp[(int64_t)k0 * ldb + e];
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 4; ++e) As[buf][ak + e][ar] = ra[e];
#pragma unroll
    for (int e = 0; e < 4; ++e) Bs[buf][bk][bn + e] = rb[e];
  };

  V4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = V4{0, 0, 0, 0};

  const int lr = lane & 15, lk = lane >> 4;
  fetch(0);
  stash(0);
  __syncthreads();
  const int nk = K / BK;
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) fetch((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      T a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[buf][kk * 4 + lk][wm * 32 + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[buf][kk * 4 + lk][wn * 32 + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = Acc<T>::mfma(a[i], b[j], acc[i][j]);
    }
    if (kt + 1 < nk) stash(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn * 32 + j * 16 + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 32 + i * 16 + Acc<T>::row(lk, v);
        if (row < M) C[(int64_t)row * ldc + col] = acc[i][j][v];
      }
    }
  }
}

template <typename T>
hipError_t gemm_launch(const T* A, int64_t sA, int lda, const T* B, int64_t sB, int ldb, T* C,
                       int64_t sC, int ldc, int M, int N, int K, int batch, hipStream_t s) {
  if (N % BN || K % BK || M <= 0 || batch <= 0) return hipErrorInvalidValue;
  const int tiles_m = (M + BM - 1) / BM, tiles_n = N / BN;
  const int64_t nblk = (int64_t)tiles_m * tiles_n * batch;
  if (nblk > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_gemm<T>), dim3((unsigned)nblk), dim3(GTHREADS), 0, s, A, sA, lda, B, sB,
                     ldb, C, sC, ldc, M, N, K, tiles_m, tiles_n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- shifted divide
template <typename T>
__global__ void k_divide(T* __restrict__ spec, const double* __restrict__ lam,
                         const double* __restrict__ tmu1, const double* __restrict__ tmu2,
                         const double* __restrict__ tmu3, int nh, int m1, int m2, int m3, int P1,
                         int P2, int64_t PS) {
  const int64_t total = (int64_t)nh * PS;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(idx / PS);
    const int64_t p = idx - (int64_t)k * PS;
    const int i1 = (int)(p % P1);
    const int64_t q = p / P1;
    const int i2 = (int)(q % P2);
    const int i3 = (int)(q / P2);
    T* re = spec + (int64_t)k * 2 * PS + p;
    T* im = re + PS;
    if (i1 >= m1 || i2 >= m2 || i3 >= m3) {
      *re = T(0);
      *im = T(0);
      continue;
    }
    const T c = (T)(lam[2 * k] + tmu1[i1] + (tmu2 ? tmu2[i2] : 0.0) + (tmu3 ? tmu3[i3] : 0.0));
    const T d = (T)lam[2 * k + 1];
    const T a = *re, b = *im;
    const T inv = T(1) / (c * c + d * d);
    *re = (a * c + b * d) * inv;
    *im = (b * c - a * d) * inv;
  }
}

// ---------------------------------------------------------------- layout conversion
template <typename T>
__global__ void k_spec_to_ext(const T* __restrict__ spec, double* __restrict__ ext, int nh,
                              int m1, int m2, int m3, int P1, int P2, int64_t PS) {
  const int64_t m = (int64_t)m1 * m2 * m3;
  const int64_t total = (int64_t)nh * m;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(idx / m);
    const int64_t s = idx - (int64_t)k * m;
    const int i1 = (int)(s % m1);
    const int64_t q = s / m1;
    const int i2 = (int)(q % m2);
    const int i3 = (int)(q / m2);
    const int64_t p = ((int64_t)i3 * P2 + i2) * P1 + i1;
    const T* re = spec + (int64_t)k * 2 * PS + p;
    ext[2 * idx] = (double)re[0];
    ext[2 * idx + 1] = (double)re[PS];
  }
}

template <typename T>
__global__ void k_ext_to_spec(const double* __restrict__ ext, T* __restrict__ spec, int nh,
                              int m1, int m2, int m3, int P1, int P2, int64_t PS) {
  // writes every position of every plane: data where valid, zero in padding
  const int64_t total = (int64_t)nh * PS;
  const int64_t m = (int64_t)m1 * m2 * m3;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(idx / PS);
    const int64_t p = idx - (int64_t)k * PS;
    const int i1 = (int)(p % P1);
    const int64_t q = p / P1;
    const int i2 = (int)(q % P2);
    const int i3 = (int)(q / P2);
    T* re = spec + (int64_t)k * 2 * PS + p;
    if (i1 >= m1 || i2 >= m2 || i3 >= m3) {
      re[0] = T(0);
      re[PS] = T(0);
      continue;
    }
    const int64_t s = ((int64_t)i3 * m2 + i2) * m1 + i1;
    const double* e = ext + 2 * ((int64_t)k * m + s);
    re[0] = (T)e[0];
    re[PS] = (T)e[1];
  }
}

unsigned grid_for(int64_t total, int threads) {
  int64_t b = (total + threads - 1) / threads;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_gemm_f64(const double* A, int64_t sA, int lda, const double* B, int64_t sB,
                           int ldb, double* C, int64_t sC, int ldc, int M, int N, int K,
                           int batch, hipStream_t s) {
  return gemm_launch<double>(A, sA, lda, B, sB, ldb, C, sC, ldc, M, N, K, batch, s);
}
hipError_t launch_gemm_f32(const float* A, int64_t sA, int lda, const float* B, int64_t sB,
                           int ldb, float* C, int64_t sC, int ldc, int M, int N, int K, int batch,
                           hipStream_t s) {
  return gemm_launch<float>(A, sA, lda, B, sB, ldb, C, sC, ldc, M, N, K, batch, s);
}

hipError_t launch_divide_f64(const Geometry& g, double* spec, const double* lam,
                             const double* tmu1, const double* tmu2, const double* tmu3,
                             hipStream_t s) {
  hipLaunchKernelGGL((k_divide<double>), dim3(grid_for((int64_t)g.nh * g.PS, 256)), dim3(256), 0,
                     s, spec, lam, tmu1, tmu2, tmu3, g.nh, g.m1, g.m2, g.m3, g.P1, g.P2, g.PS);
  return hipGetLastError();
}
hipError_t launch_divide_f32(const Geometry& g, float* spec, const double* lam,
                             const double* tmu1, const double* tmu2, const double* tmu3,
                             hipStream_t s) {
  hipLaunchKernelGGL((k_divide<float>), dim3(grid_for((int64_t)g.nh * g.PS, 256)), dim3(256), 0,
                     s, spec, lam, tmu1, tmu2, tmu3, g.nh, g.m1, g.m2, g.m3, g.P1, g.P2, g.PS);
  return hipGetLastError();
}

hipError_t launch_spec_to_ext(const Geometry& g, const void* spec, int is_f32, double* ext,
                              hipStream_t s) {
  const unsigned grid = grid_for((int64_t)g.nh * g.m, 256);
  if (is_f32)
    hipLaunchKernelGGL((k_spec_to_ext<float>), dim3(grid), dim3(256), 0, s, (const float*)spec,
                       ext, g.nh, g.m1, g.m2, g.m3, g.P1, g.P2, g.PS);
  else
    hipLaunchKernelGGL((k_spec_to_ext<double>), dim3(grid), dim3(256), 0, s,
                       (const double*)spec, ext, g.nh, g.m1, g.m2, g.m3, g.P1, g.P2, g.PS);
  return hipGetLastError();
}

hipError_t launch_ext_to_spec(const Geometry& g, const double* ext, void* spec, int is_f32,
                              hipStream_t s) {
  const unsigned grid = grid_for((int64_t)g.nh * g.PS, 256);
  if (is_f32)
    hipLaunchKernelGGL((k_ext_to_spec<float>), dim3(grid), dim3(256), 0, s, ext, (float*)spec,
                       g.nh, g.m1, g.m2, g.m3, g.P1, g.P2, g.PS);
  else
    hipLaunchKernelGGL((k_ext_to_spec<double>), dim3(grid), dim3(256), 0, s, ext, (double*)spec,
                       g.nh, g.m1, g.m2, g.m3, g.P1, g.P2, g.PS);
  return hipGetLastError();
}

}  // namespace aao
