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

  // tiles sharing an A row-block (tn fastest) stay in one XCD's L2
  int bid = xcd_remap(blockIdx.x, gridDim.x);
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

// ---------------------------------------------------------------- BF16 hi/lo products
// C = A * B with one FP32 operand (the spectrum) split on the fly into
// hi = rne_bf16(x), lo = rne_bf16(x - hi) and the other (S) split once on the
// host; C accumulates hi*hi + hi*lo + lo*hi in FP32 on v_mfma_f32_16x16x32_bf16.
// Both LDS tiles keep k contiguous so that each lane reads its 8 k values of
// a fragment with one 16-byte load.  With the data on the right (B = data
// rows of k) the B tile is stored transposed, one 16-bit element per store,
// by lanes that hold 8 consecutive columns: with
// rows 20 dwords apart the 8 column groups of a wave would all hit the same 4
// banks, so its 16-byte k chunks are XOR-swizzled by column group
// (chunk (k/8) ^ ((n/8) & 3)), which leaves the fragment reads of 8 lanes
// (one column group) conflict-free and spreads the stores over 16 banks.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s8v __attribute__((ext_vector_type(8)));
typedef unsigned short u16;

__device__ __forceinline__ u16 bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}
__device__ __forceinline__ float bf16_val(u16 h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int XBK = 32, XPAD = 8;

template <bool A_DATA>
__global__ __launch_bounds__(GTHREADS) void k_gemm_bf16x3(
    const float* __restrict__ Dm, int64_t sD, int ldd,          // FP32 data operand
    const u16* __restrict__ Shi, const u16* __restrict__ Slo,   // pre-split operand
    int lds_, float* __restrict__ C, int64_t sC, int ldc, int M, int N, int K, int tiles_m,
    int tiles_n) {
  __shared__ __attribute__((aligned(16))) u16 Ah[2][BM][XBK + XPAD];
  __shared__ __attribute__((aligned(16))) u16 Al[2][BM][XBK + XPAD];
  __shared__ __attribute__((aligned(16))) u16 Bh[2][BN][XBK + XPAD];
  __shared__ __attribute__((aligned(16))) u16 Bl[2][BN][XBK + XPAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int bid = blockIdx.x;
  const int tn = bid % tiles_n;
  bid /= tiles_n;
  const int tm = bid % tiles_m;
  const int batch = bid / tiles_m;
  const int m0 = tm * BM, n0 = tn * BN;
  Dm += batch * sD;
  C += batch * sC;

  // A tile: row ar (0..63), k ak..ak+7;  B tile: k bk (0..31), cols bn..bn+7
  const int ar = tid >> 2, ak = (tid & 3) * 8;
  const int bk = tid >> 3, bn = (tid & 7) * 8;
  const bool arow_ok = (m0 + ar) < M;

  u16 rah[8], ral[8], rbh[8], rbl[8];
  auto fetch = [&](int k0) {
    if (A_DATA) {  // A = data rows (M x K, ldd), B = S (K x N, lds_)
      // 8 consecutive k of one row: two 16-byte loads (the launcher checks
      // that the data pointer, ldd and the batch stride keep them aligned)
      const float4* p = reinterpret_cast<const float4*>(
          Dm + (int64_t)(arow_ok ? m0 + ar : 0) * ldd + k0 + ak);
      const float4 q0 = p[0], q1 = p[1];
      const float xv[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float x = arow_ok ? xv[e] : 0.f;
        rah[e] = bf16_rne(x);
        ral[e] = bf16_rne(x - bf16_val(rah[e]));
      }
      // S is symmetric (the DST-I matrix), so B[k][n] = S[n][k]: 8 consecutive
      // k of column n are one 16-byte run of row n
      const int64_t o = (int64_t)(n0 + ar) * lds_ + k0 + ak;
#pragma unroll
      for (int e = 0; e < 8; ++e) { rbh[e] = Shi[o + e]; rbl[e] = Slo[o + e]; }
    } else {       // A = S (M x K, lds_), B = data (K x N, ldd)
      const int64_t o = (int64_t)(m0 + ar) * lds_ + k0 + ak;
#pragma unroll
      for (int e = 0; e < 8; ++e) { rah[e] = Shi[o + e]; ral[e] = Slo[o + e]; }
      const float* p = Dm + (int64_t)(k0 + bk) * ldd + n0 + bn;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float x = p[e];
        rbh[e] = bf16_rne(x);
        rbl[e] = bf16_rne(x - bf16_val(rbh[e]));
      }
    }
  };
  // swizzled position of k in the B tile row of column n (16-byte chunks permuted)
  auto bsw = [](int n, int k) { return (((k >> 3) ^ ((n >> 3) & 3)) << 3) | (k & 7); };
  auto stash = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 8; ++e) { Ah[buf][ar][ak + e] = rah[e]; Al[buf][ar][ak + e] = ral[e]; }
    if (A_DATA) {   // column ar, k chunk ak: one 16-byte store at its swizzled chunk
      const int bks = bsw(ar, ak);
#pragma unroll
      for (int e = 0; e < 8; ++e) { Bh[buf][ar][bks + e] = rbh[e]; Bl[buf][ar][bks + e] = rbl[e]; }
    } else {        // 8 columns of one k: transposed, one element per store
      const int bks = bsw(bn, bk);   // bn + e shares bn's column group
#pragma unroll
      for (int e = 0; e < 8; ++e) { Bh[buf][bn + e][bks] = rbh[e]; Bl[buf][bn + e][bks] = rbl[e]; }
    }
  };

  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0, 0, 0, 0};

  const int lr = lane & 15, lk = lane >> 4;
  fetch(0);
  stash(0);
  __syncthreads();
  const int nk = K / XBK;
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) fetch((kt + 1) * XBK);
    bf16x8 ahi[2], alo[2], bhi[2], blo[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int r = wm * 32 + i * 16 + lr;
      ahi[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const s8v*>(&Ah[buf][r][lk * 8]));
      alo[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const s8v*>(&Al[buf][r][lk * 8]));
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = wn * 32 + j * 16 + lr, kc = bsw(c, lk * 8);
      bhi[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const s8v*>(&Bh[buf][c][kc]));
      blo[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const s8v*>(&Bl[buf][c][kc]));
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[i], bhi[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[i], blo[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[i], bhi[j], acc[i][j], 0, 0, 0);
      }
    if (kt + 1 < nk) stash(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn * 32 + j * 16 + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 32 + i * 16 + 4 * lk + v;
        if (row < M) C[(int64_t)row * ldc + col] = acc[i][j][v];
      }
    }
}

template <bool A_DATA>
hipError_t bf16x3_launch(const float* D, int64_t sD, int ldd, const u16* Shi, const u16* Slo,
                         int lds_, float* C, int64_t sC, int ldc, int M, int N, int K, int batch,
                         hipStream_t s) {
  if (N % BN || K % XBK || M <= 0 || batch <= 0) return hipErrorInvalidValue;
  if (!A_DATA && M % BM) return hipErrorInvalidValue;
  if (A_DATA && (reinterpret_cast<uintptr_t>(D) % 16 || ldd % 4 || sD % 4))
    return hipErrorInvalidValue;   // the data rows are read 16 bytes at a time
  const int tiles_m = (M + BM - 1) / BM, tiles_n = N / BN;
  const int64_t nblk = (int64_t)tiles_m * tiles_n * batch;
  if (nblk > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_gemm_bf16x3<A_DATA>), dim3((unsigned)nblk), dim3(GTHREADS), 0, s, D, sD,
                     ldd, Shi, Slo, lds_, C, sC, ldc, M, N, K, tiles_m, tiles_n);
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

hipError_t launch_gemm_bf16x3(const uint16_t* Ahi, const uint16_t* Alo, int64_t sA, int lda,
                              const float* B, int64_t sB, int ldb, float* C, int64_t sC, int ldc,
                              int M, int N, int K, int batch, hipStream_t s) {
  if (sA != 0) return hipErrorInvalidValue;  // the split operand is a shared matrix
  return bf16x3_launch<false>(B, sB, ldb, Ahi, Alo, lda, C, sC, ldc, M, N, K, batch, s);
}

// B must be symmetric (the kernel reads B[k][n] as B[n][k]); lda = ldb = K = N.
hipError_t launch_gemm_bf16x3_right(const float* A, int64_t sA, int lda, const uint16_t* Bhi,
                                    const uint16_t* Blo, int64_t sB, int ldb, float* C,
                                    int64_t sC, int ldc, int M, int N, int K, int batch,
                                    hipStream_t s) {
  if (sB != 0 || N != K) return hipErrorInvalidValue;   // a symmetric (square) B
  return bf16x3_launch<true>(A, sA, lda, Bhi, Blo, ldb, C, sC, ldc, M, N, K, batch, s);
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
