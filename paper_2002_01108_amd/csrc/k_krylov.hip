// FP64 vector kernels of the flexible GMRES loop: multi-vector dot products
// for classical Gram-Schmidt, the fused update-then-dot/norm passes of its
// second sweep, solution update, scaling and residual norms.
//
// Reductions are deterministic: every block writes its partial sums, a second
// kernel adds the partials of each output in a fixed tree order.  Each thread
// reads two consecutive doubles per step (16-byte loads) in a grid-stride loop.
#include "common.h"

namespace aao {
namespace {

constexpr int KT = 256;        // threads per block
constexpr int QMAX = 8;        // vectors per fused pass
constexpr int MAXBLK = 8192;   // partial-sum blocks (fewer leave the streaming passes 6 % slower)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block-reduce Q accumulators; thread 0 writes part[blk*qtot + qoff + i].
template <int Q>
__device__ __forceinline__ void block_store(double (&acc)[Q], double* part, int qtot, int qoff) {
  __shared__ double red[Q][KT / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double v = wave_sum(acc[i]);
    if (lane == 0) red[i][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < Q) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < KT / 64; ++w) s += red[threadIdx.x][w];
    part[(int64_t)blockIdx.x * qtot + qoff + threadIdx.x] = s;
  }
}

// Basis vector i: V + i*ldv, except vector 0 which is v0 when v0 is non-null
// (the Krylov basis may start from a caller's array without a copy).
__device__ __forceinline__ const double* basis(const double* V, int64_t ldv, const double* v0,
                                               int i) {
  return (i == 0 && v0) ? v0 : V + i * ldv;
}

// part[b*qtot + qoff + i] = partial sum of V_{qoff+i} . w
template <int Q>
__global__ __launch_bounds__(KT) void k_multidot(const double* __restrict__ V, int64_t ldv,
                                                 const double* __restrict__ v0,
                                                 const double* __restrict__ w, int64_t len,
                                                 double* __restrict__ part, int qtot, int qoff) {
  double acc[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) acc[i] = 0.0;
  const int64_t npair = len >> 1;
  const double2* w2 = reinterpret_cast<const double2*>(w);
  for (int64_t e = blockIdx.x * (int64_t)KT + threadIdx.x; e < npair;
       e += (int64_t)gridDim.x * KT) {
    const double2 wv = w2[e];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double2 v = reinterpret_cast<const double2*>(basis(V, ldv, v0, qoff + i))[e];
      acc[i] += v.x * wv.x + v.y * wv.y;
    }
  }
  if ((len & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < Q; ++i) acc[i] += basis(V, ldv, v0, qoff + i)[len - 1] * w[len - 1];
  }
  block_store<Q>(acc, part, qtot, qoff);
}

// w -= sum_{i<q} h_i V_i; then MODE 1: partial dots of V_0..V_{Q-1} with the
// new w (requires q == Q) into part[b*Q + i] and its partial squared norm into
// part[gridDim.x*Q + b];  MODE 2: partial ||w||^2;  MODE 0: nothing.
template <int Q, int MODE>
__global__ __launch_bounds__(KT) void k_axpy(const double* __restrict__ V, int64_t ldv,
                                             const double* __restrict__ v0, int q,
                                             const double* __restrict__ h, double* __restrict__ w,
                                             int64_t len, double* __restrict__ part) {
  double acc[Q];
  double nrm[1] = {0.0};
#pragma unroll
  for (int i = 0; i < Q; ++i) acc[i] = 0.0;
  const int64_t npair = len >> 1;
  double2* w2 = reinterpret_cast<double2*>(w);
  auto body = [&](double& wx, int64_t idx) {
    // scalar element update (used for the odd tail)
    double s = wx;
    for (int i = 0; i < q; ++i) s -= h[i] * basis(V, ldv, v0, i)[idx];
    wx = s;
    if (MODE == 1) {
#pragma unroll
      for (int i = 0; i < Q; ++i) acc[i] += basis(V, ldv, v0, i)[idx] * s;
      nrm[0] += s * s;
    } else if (MODE == 2) {
      acc[0] += s * s;
    }
  };
  const int64_t gs = (int64_t)gridDim.x * KT;
  int64_t e0 = blockIdx.x * (int64_t)KT + threadIdx.x;
  if (MODE == 1 && Q == 1) {
    // the Gram-Schmidt pass of an Arnoldi step with one basis vector: two
    // element pairs per iteration, all loads issued before the arithmetic, in
    // the same element order per thread as the loop below (2.73 -> 2.58 ms at
    // 127^3 x 256)
    const double h0 = h[0];
    const double2* b0 = reinterpret_cast<const double2*>(basis(V, ldv, v0, 0));
    for (; e0 + gs < npair; e0 += 2 * gs) {
      const int64_t e1 = e0 + gs;
      double2 wa = w2[e0], wb = w2[e1];
      const double2 va = b0[e0], vb = b0[e1];
      wa.x -= h0 * va.x; wa.y -= h0 * va.y;
      wb.x -= h0 * vb.x; wb.y -= h0 * vb.y;
      w2[e0] = wa;
      w2[e1] = wb;
      acc[0] += va.x * wa.x + va.y * wa.y;
      nrm[0] += wa.x * wa.x + wa.y * wa.y;
      acc[0] += vb.x * wb.x + vb.y * wb.y;
      nrm[0] += wb.x * wb.x + wb.y * wb.y;
    }
  }
  for (int64_t e = e0; e < npair; e += gs) {
    double2 wv = w2[e];
    for (int i = 0; i < q; ++i) {
      const double hi = h[i];
      const double2 v = reinterpret_cast<const double2*>(basis(V, ldv, v0, i))[e];
      wv.x -= hi * v.x;
      wv.y -= hi * v.y;
    }
    w2[e] = wv;
    if (MODE == 1) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const double2 v = reinterpret_cast<const double2*>(basis(V, ldv, v0, i))[e];
        acc[i] += v.x * wv.x + v.y * wv.y;
      }
      nrm[0] += wv.x * wv.x + wv.y * wv.y;
    } else if (MODE == 2) {
      acc[0] += wv.x * wv.x + wv.y * wv.y;
    }
  }
  if ((len & 1) && blockIdx.x == 0 && threadIdx.x == 0) body(w[len - 1], len - 1);
  if (MODE != 0) block_store<Q>(acc, part, MODE == 1 ? Q : 1, 0);
  if (MODE == 1) {
    __syncthreads();   // block_store's LDS is reused
    block_store<1>(nrm, part + (int64_t)gridDim.x * Q, 1, 0);
  }
}

// out[i] (+)= scale_i * sum_b part[b*q + i] (scale_i = 1 when scale is null),
// one block per output
__global__ __launch_bounds__(KT) void k_reduce(const double* __restrict__ part, int nblk, int q,
                                               double* __restrict__ out, int accumulate,
                                               const double* __restrict__ scale) {
  const int i = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += KT) s += part[(int64_t)b * q + i];
  __shared__ double red[KT / 64];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < KT / 64; ++w) t += red[w];
    if (scale) t *= scale[i];
    out[i] = accumulate ? out[i] + t : t;
  }
}

__global__ void k_scale(const double* __restrict__ x, double* __restrict__ y, int64_t len,
                        double a) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x)
    y[e] = a * x[e];
}

// x (+)= sum_i c_i Z_i; with set != 0 x is overwritten (not read)
__global__ void k_multi_axpy(const double* __restrict__ Z, int64_t ldz, int q,
                             const double* __restrict__ c, double* __restrict__ x, int64_t len,
                             int set) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = set ? 0.0 : x[e];
    for (int i = 0; i < q; ++i) s += c[i] * Z[i * ldz + e];
    x[e] = s;
  }
}

// The same for Q <= 4 vectors known at compile time, two elements per thread
// and access (Z, x and the row stride 16-byte aligned): all loads of an element
// pair are issued together.  Same summation order as k_multi_axpy.
template <int Q>
__global__ void k_multi_axpy2(const double* __restrict__ Z, int64_t ldz,
                              const double* __restrict__ c, double* __restrict__ x, int64_t len,
                              int set) {
  double ci[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) ci[i] = c[i];
  const int64_t npair = len >> 1;
  double2* x2 = reinterpret_cast<double2*>(x);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < npair;
       e += (int64_t)gridDim.x * blockDim.x) {
    double2 z[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) z[i] = reinterpret_cast<const double2*>(Z + i * ldz)[e];
    double2 s = set ? double2{0.0, 0.0} : x2[e];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      s.x += ci[i] * z[i].x;
      s.y += ci[i] * z[i].y;
    }
    x2[e] = s;
  }
  if ((len & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    double s = set ? 0.0 : x[len - 1];
#pragma unroll
    for (int i = 0; i < Q; ++i) s += ci[i] * Z[i * ldz + len - 1];
    x[len - 1] = s;
  }
}

// part[b] = partial ||a - b||^2 (b null -> ||a||^2); non-finite values propagate
__global__ __launch_bounds__(KT) void k_diffnorm(const double* __restrict__ a,
                                                 const double* __restrict__ b, int64_t len,
                                                 double* __restrict__ part) {
  double acc[1] = {0.0};
  for (int64_t e = blockIdx.x * (int64_t)KT + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * KT) {
    const double d = b ? a[e] - b[e] : a[e];
    acc[0] += d * d;
  }
  block_store<1>(acc, part, 1, 0);
}

__global__ void k_build_rhs(const double* __restrict__ f, const double* __restrict__ u0,
                            double* __restrict__ y, int64_t nm, int64_t m, double tau,
                            double r2) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nm;
       e += (int64_t)gridDim.x * blockDim.x) {
    double v = tau * f[e];
    if (e < m) v += u0[e];
    else if (r2 != 0.0 && e < 2 * m) v -= r2 * u0[e - m];
    y[e] = v;
  }
}

// One thread per (time level, row): the west and east boundary terms of the
// row, and for the first / last row also the south / north terms of each
// column, so no two threads touch the same entry.
__global__ void k_boundary_source(const double* __restrict__ gb, const double* __restrict__ cb,
                                  double* __restrict__ f, int n, int m1, int m2) {
  const int64_t nb = 2LL * m1 + 2LL * m2;
  const int64_t total = (int64_t)n * m2;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(e / m2), j = (int)(e - (int64_t)k * m2);
    const double* g = gb + k * nb;
    double* row = f + ((int64_t)k * m2 + j) * m1;
    row[0] += cb[j] * g[j];
    row[m1 - 1] += cb[m2 + j] * g[m2 + j];
    if (j == 0)
      for (int i = 0; i < m1; ++i) row[i] += cb[2 * m2 + i] * g[2 * m2 + i];
    if (j == m2 - 1)
      for (int i = 0; i < m1; ++i) row[i] += cb[2 * m2 + m1 + i] * g[2 * m2 + m1 + i];
  }
}

unsigned simple_grid(int64_t len) {
  int64_t b = (len + 255) / 256;
  if (b > 16384) b = 16384;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

int krylov_blocks(int64_t len) {
  int64_t b = ((len >> 1) + KT * 4 - 1) / (KT * 4);
  if (b > MAXBLK) b = MAXBLK;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_multidot(const double* V, int64_t ldv, const double* v0, int q,
                           const double* w, int64_t len, double* part, hipStream_t s) {
  const int nb = krylov_blocks(len);
  for (int q0 = 0; q0 < q; q0 += QMAX) {
    const int qq = (q - q0 < QMAX) ? q - q0 : QMAX;
    switch (qq) {
#define CASE(Q)                                                                                \
  case Q:                                                                                      \
    hipLaunchKernelGGL((k_multidot<Q>), dim3(nb), dim3(KT), 0, s, V, ldv, v0, w, len, part, q, \
                       q0);                                                                    \
    break;
      CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    }
  }
  return hipGetLastError();
}

hipError_t launch_axpy_dot(const double* V, int64_t ldv, const double* v0, int q,
                           const double* h, double* w, int64_t len, double* part, int mode,
                           hipStream_t s) {
  const int nb = krylov_blocks(len);
  if (mode == 1) {
    if (q > QMAX || q < 1) return hipErrorInvalidValue;
    switch (q) {
#define CASE(Q)                                                                             \
  case Q:                                                                                   \
    hipLaunchKernelGGL((k_axpy<Q, 1>), dim3(nb), dim3(KT), 0, s, V, ldv, v0, q, h, w, len,    \
                       part);                                                                 \
    break;
      CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    }
  } else if (mode == 2) {
    hipLaunchKernelGGL((k_axpy<1, 2>), dim3(nb), dim3(KT), 0, s, V, ldv, v0, q, h, w, len, part);
  } else {
    hipLaunchKernelGGL((k_axpy<1, 0>), dim3(nb), dim3(KT), 0, s, V, ldv, v0, q, h, w, len, part);
  }
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* part, int nblk, int q, double* out, int accumulate,
                                  const double* scale, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(q), dim3(KT), 0, s, part, nblk, q, out, accumulate, scale);
  return hipGetLastError();
}

hipError_t launch_scale_host(const double* x, double* y, int64_t len, double alpha,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(simple_grid(len)), dim3(256), 0, s, x, y, len, alpha);
  return hipGetLastError();
}

hipError_t launch_multi_axpy(const double* Z, int64_t ldz, int q, const double* c, double* x,
                             int64_t len, int set, hipStream_t s) {
  const bool vec = q >= 1 && q <= 4 && ((uintptr_t)Z % 16 == 0) && ((uintptr_t)x % 16 == 0) &&
                   (ldz % 2 == 0);
  if (vec) {
    const unsigned g = simple_grid((len + 1) / 2);
    switch (q) {
      case 1:
        hipLaunchKernelGGL((k_multi_axpy2<1>), dim3(g), dim3(256), 0, s, Z, ldz, c, x, len, set);
        break;
      case 2:
        hipLaunchKernelGGL((k_multi_axpy2<2>), dim3(g), dim3(256), 0, s, Z, ldz, c, x, len, set);
        break;
      case 3:
        hipLaunchKernelGGL((k_multi_axpy2<3>), dim3(g), dim3(256), 0, s, Z, ldz, c, x, len, set);
        break;
      default:
        hipLaunchKernelGGL((k_multi_axpy2<4>), dim3(g), dim3(256), 0, s, Z, ldz, c, x, len, set);
        break;
    }
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_multi_axpy, dim3(simple_grid(len)), dim3(256), 0, s, Z, ldz, q, c, x, len,
                     set);
  return hipGetLastError();
}

hipError_t launch_diffnorm(const double* a, const double* b, int64_t len, double* part,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_diffnorm, dim3(krylov_blocks(len)), dim3(KT), 0, s, a, b, len, part);
  return hipGetLastError();
}

hipError_t launch_build_rhs(const double* f, const double* u0, double* y, int64_t nm, int64_t m,
                            double tau, double r2, hipStream_t s) {
  hipLaunchKernelGGL(k_build_rhs, dim3(simple_grid(nm)), dim3(256), 0, s, f, u0, y, nm, m, tau,
                     r2);
  return hipGetLastError();
}

hipError_t launch_boundary_source(const double* gb, const double* cb, double* f, int n, int m1,
                                  int m2, hipStream_t s) {
  if (n < 1 || m1 < 1 || m2 < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_boundary_source, dim3(simple_grid((int64_t)n * m2)), dim3(256), 0, s, gb,
                     cb, f, n, m1, m2);
  return hipGetLastError();
}

}  // namespace aao
