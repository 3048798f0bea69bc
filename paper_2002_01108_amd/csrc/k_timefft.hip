// Steps 1 and 3 of the BEC inverse (Section 4, eqs. (ytild) and (zcompt)):
//   Step 1: ytilde^{k} = n^{-1/2} sum_j theta^{kj} eps^{j/n} y^{j},  k = 0..n/2
//   Step 3: z^{j}     = eps^{-j/n} n^{-1/2} sum_k theta^{-kj} ztilde^{k}
// with theta = exp(+2 pi i/n) (eq. (fouriermatdef)) and ztilde^{n-k} =
// conj(ztilde^k) (conjugate symmetry at the end of Section 4).
//
// The transform runs along time, the slowest axis of the [n][m] array.  A
// block owns 2 CW consecutive spatial points of one x-row (paired as c and
// c + CW) and all n time levels: consecutive lanes read consecutive addresses
// of each time row, every load and store instruction is contiguous.  Two
// real sequences a, b travel as one complex sequence a + i b ("two for one"),
// untangled after the forward transform and re-tangled before the inverse.
// The FFT is a Stockham autosort sequence of radix-16 (last: smaller) passes;
// each thread keeps its butterfly's points in registers and the passes
// exchange through one LDS tile of n x CW complex values.  The first pass of
// both kernels and the last pass of the inverse go straight to HBM.
//
// Output of Step 1 (input of Step 3) is the split-plane spectrum layout:
//   spec[k][0][i3][i2][i1] = Re, spec[k][1][i3][i2][i1] = Im, planes padded to
//   P1 x P2 x P3; Step 1 writes zeros into every padding position it covers.
#include "common.h"

namespace aao {
namespace {

// TH threads per block: 256, or 512 for long transforms of HBM-resident data
// (wider column strips per block keep more of each DRAM page per request).
template <int N, int TH> struct Cfg {
  static constexpr int R1 = N < 16 ? N : 16;
  static constexpr int TPC = N / R1;     // threads per column
  static constexpr int CW = TH / TPC;    // complex columns per block
};

// multiply by exp(SIGN * 2 pi i * e / 16) for a compile-time-known e in [0,16)
template <typename T, int SIGN>
__device__ __forceinline__ cplx<T> rot16(int e, cplx<T> d) {
  const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);
  const T h = T(0.70710678118654752440);
  T cs, sn;
  switch (e & 15) {
    case 0: return d;
    case 4: return SIGN > 0 ? cplx<T>{-d.y, d.x} : cplx<T>{d.y, -d.x};
    case 8: return {-d.x, -d.y};
    case 12: return SIGN > 0 ? cplx<T>{d.y, -d.x} : cplx<T>{-d.y, d.x};
    case 1: cs = c1; sn = s1; break;
    case 2: cs = h; sn = h; break;
    case 3: cs = s1; sn = c1; break;
    case 5: cs = -s1; sn = c1; break;
    case 6: cs = -h; sn = h; break;
    case 7: cs = -c1; sn = s1; break;
    case 9: cs = -c1; sn = -s1; break;
    case 10: cs = -h; sn = -h; break;
    case 11: cs = -s1; sn = -c1; break;
    case 13: cs = s1; sn = -c1; break;
    case 14: cs = h; sn = -h; break;
    default: cs = c1; sn = -s1; break;  // 15
  }
  if (SIGN < 0) sn = -sn;
  return {d.x * cs - d.y * sn, d.x * sn + d.y * cs};
}

// In-register DFT of length R (power of two <= 16), X[k] = sum_j v[j] w^{jk},
// w = exp(SIGN 2 pi i / R), natural order in and out.  Radix-2 decimation in
// frequency followed by the bit-reversal permutation (register renaming).
template <typename T, int R, int SIGN>
__device__ __forceinline__ void dft(cplx<T>* v) {
  if constexpr (R == 1) {
    return;
  } else {
#pragma unroll
    for (int half = R / 2; half >= 1; half >>= 1) {
#pragma unroll
      for (int b = 0; b < R; b += 2 * half) {
#pragma unroll
        for (int i = 0; i < half; ++i) {
          const cplx<T> a = v[b + i], c = v[b + i + half];
          v[b + i] = cadd(a, c);
          v[b + i + half] = rot16<T, SIGN>(i * (R / (2 * half)) * (16 / R), csub(a, c));
        }
      }
    }
    cplx<T> tmp[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      int r = 0;
#pragma unroll
      for (int bit = 1, rb = R / 2; bit < R; bit <<= 1, rb >>= 1)
        if (k & bit) r |= rb;
      tmp[k] = v[r];
    }
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = tmp[k];
  }
}

template <typename T, int SIGN>
__device__ __forceinline__ cplx<T> twiddle(const cplx<T>* __restrict__ tw, int e, cplx<T> d) {
  cplx<T> w = tw[e];
  if (SIGN < 0) w.y = -w.y;
  return cmul(d, w);
}

// One Stockham pass (accumulated length NS -> NS*R) from the LDS tile.
// Results go back to LDS unless FINAL, in which case sink(index, value) gets them.
template <typename T, int N, int TH, int SIGN, int NS, bool FINAL, typename Sink>
__device__ __forceinline__ void lds_pass(cplx<T>* lds, const cplx<T>* __restrict__ tw, int t,
                                         int c, Sink&& sink) {
  using C = cplx<T>;
  constexpr int TPC = Cfg<N, TH>::TPC, CW = Cfg<N, TH>::CW;
  constexpr int R = (N / NS) < 16 ? (N / NS) : 16;
  constexpr int NB = N / R;
  constexpr int PER = NB / TPC;
  C v[PER][R];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = t + q * TPC;
    const int e = (j % NS) * (N / (NS * R));
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const C d = lds[(j + r * NB) * CW + c];
      v[q][r] = (r == 0) ? d : twiddle<T, SIGN>(tw, (r * e) & (N - 1), d);
    }
  }
  if constexpr (!FINAL) __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = t + q * TPC;
    dft<T, R, SIGN>(v[q]);
    const int idxD = (j / NS) * NS * R + (j % NS);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if constexpr (FINAL)
        sink(idxD + r * NS, v[q][r]);
      else
        lds[(idxD + r * NS) * CW + c] = v[q][r];
    }
  }
}

// All passes after the first, writing back to LDS, ending with a barrier.
template <typename T, int N, int TH, int SIGN, int NS>
__device__ __forceinline__ void lds_passes_all(cplx<T>* lds, const cplx<T>* __restrict__ tw, int t,
                                               int c) {
  if constexpr (NS < N) {
    lds_pass<T, N, TH, SIGN, NS, false>(lds, tw, t, c, [](int, cplx<T>) {});
    constexpr int R = (N / NS) < 16 ? (N / NS) : 16;
    lds_passes_all<T, N, TH, SIGN, NS * R>(lds, tw, t, c);
  } else {
    __syncthreads();
  }
}

// Passes after the first except the last (which the caller runs as FINAL).
template <typename T, int N, int TH, int SIGN, int NS>
__device__ __forceinline__ void lds_passes_but_last(cplx<T>* lds, const cplx<T>* __restrict__ tw,
                                                    int t, int c) {
  constexpr int R = (N / NS) < 16 ? (N / NS) : 16;
  if constexpr (NS * R < N) {
    lds_pass<T, N, TH, SIGN, NS, false>(lds, tw, t, c, [](int, cplx<T>) {});
    lds_passes_but_last<T, N, TH, SIGN, NS * R>(lds, tw, t, c);
  }
}

template <int N, int NS> struct LastNS {
  static constexpr int R = (N / NS) < 16 ? (N / NS) : 16;
  static constexpr int value = (NS * R >= N) ? NS : LastNS<N, (NS * R >= N ? N : NS * R)>::value;
};
template <int N> struct LastNS<N, N> { static constexpr int value = N; };

// ---------------------------------------------------------------- forward (Step 1)
template <typename T, int N, int TH>
__global__ __launch_bounds__(TH) void k_time_fwd(
    const double* __restrict__ x, T* __restrict__ spec, const T* __restrict__ gam,
    const cplx<T>* __restrict__ tw, int m1, int m2, int m3, int P1, int P2, int64_t PS,
    int nseg) {
  using C = cplx<T>;
  constexpr int R1 = Cfg<N, TH>::R1, TPC = Cfg<N, TH>::TPC, CW = Cfg<N, TH>::CW;
  __shared__ C lds[N * CW];
  const int tid = threadIdx.x;
  const int c = tid % CW, t = tid / CW;
  // neighbouring column segments share cache lines: keep them in one XCD
  int b = xcd_remap(blockIdx.x, gridDim.x);
  const int sg = b % nseg;
  b /= nseg;
  const int i2 = b % P2;
  const int i3 = b / P2;
  // the two real columns of complex column c are i1a and i1a + CW, so every
  // load and store instruction of a wave covers contiguous addresses
  const int i1a = sg * 2 * CW + c, i1b = i1a + CW;
  const bool rowvalid = (i2 < m2) && (i3 < m3);
  const bool va = rowvalid && i1a < m1;
  const bool vb = rowvalid && i1b < m1;
  const int64_t m = (int64_t)m1 * m2 * m3;
  const int64_t xoff = rowvalid ? ((int64_t)i3 * m2 + i2) * m1 + i1a : 0;
  const int64_t poff = ((int64_t)i3 * P2 + i2) * P1;

  C v[R1];
#pragma unroll
  for (int r = 0; r < R1; ++r) {
    const int j = t + r * TPC;
    const double* xp = x + (int64_t)j * m + xoff;
    const T a = va ? (T)xp[0] : T(0);
    const T bb = vb ? (T)xp[CW] : T(0);
    const T gj = gam[j];
    v[r] = {a * gj, bb * gj};
  }
  dft<T, R1, +1>(v);
#pragma unroll
  for (int r = 0; r < R1; ++r) lds[(t * R1 + r) * CW + c] = v[r];
  lds_passes_all<T, N, TH, +1, R1>(lds, tw, t, c);

  // untangle: A(k) = (C(k) + conj C(n-k))/2, B(k) = (C(k) - conj C(n-k))/(2i)
  for (int k = t; k <= N / 2; k += TPC) {
    const C ck = lds[k * CW + c];
    const C cn = lds[((N - k) & (N - 1)) * CW + c];
    const T half = T(0.5);
    T* pr = spec + (int64_t)k * 2 * PS + poff;
    T* pi = pr + PS;
    if (i1a < P1) {
      pr[i1a] = va ? (ck.x + cn.x) * half : T(0);
      pi[i1a] = va ? (ck.y - cn.y) * half : T(0);
    }
    if (i1b < P1) {
      pr[i1b] = vb ? (ck.y + cn.y) * half : T(0);
      pi[i1b] = vb ? (cn.x - ck.x) * half : T(0);
    }
  }
}

// ---------------------------------------------------------------- inverse (Step 3)
template <typename T, int N, int TH>
__global__ __launch_bounds__(TH) void k_time_inv(
    const T* __restrict__ spec, double* __restrict__ z, const T* __restrict__ ginv,
    const cplx<T>* __restrict__ tw, int m1, int m2, int m3, int P1, int P2, int64_t PS,
    int nseg) {
  using C = cplx<T>;
  constexpr int R1 = Cfg<N, TH>::R1, TPC = Cfg<N, TH>::TPC, CW = Cfg<N, TH>::CW;
  __shared__ C lds[(R1 == N) ? 1 : N * CW];
  const int tid = threadIdx.x;
  const int c = tid % CW, t = tid / CW;
  // neighbouring column segments share cache lines: keep them in one XCD
  int b = xcd_remap(blockIdx.x, gridDim.x);
  const int sg = b % nseg;
  b /= nseg;
  const int i2 = b % m2;
  const int i3 = b / m2;
  const int i1a = sg * 2 * CW + c, i1b = i1a + CW;   // as in the forward kernel
  const bool va = i1a < m1;
  const bool vb = i1b < m1;
  const int64_t m = (int64_t)m1 * m2 * m3;
  const int64_t zoff = ((int64_t)i3 * m2 + i2) * m1 + i1a;
  const int64_t poff = ((int64_t)i3 * P2 + i2) * P1;

  // first pass input: C(k) = A(k) + i B(k) over the full range via A(n-k) = conj A(k)
  C v[R1];
#pragma unroll
  for (int r = 0; r < R1; ++r) {
    const int k = t + r * TPC;
    const bool upper = k > N / 2;
    const int kk = upper ? N - k : k;
    const T* pr = spec + (int64_t)kk * 2 * PS + poff;
    const T* pi = pr + PS;
    const T ar = va ? pr[i1a] : T(0);
    const T br = vb ? pr[i1b] : T(0);
    const bool realblk = (kk == 0) || (kk == N / 2);
    const T ai = (va && !realblk) ? pi[i1a] : T(0);
    const T bi = (vb && !realblk) ? pi[i1b] : T(0);
    v[r] = upper ? C{ar + bi, br - ai} : C{ar - bi, ai + br};
  }
  dft<T, R1, -1>(v);
  auto store = [&](int j, C val) {
    const T g = ginv[j];
    double* zp = z + (int64_t)j * m + zoff;
    if (va) zp[0] = (double)(val.x * g);
    if (vb) zp[CW] = (double)(val.y * g);
  };
  if constexpr (R1 == N) {
#pragma unroll
    for (int r = 0; r < R1; ++r) store(r, v[r]);  // single pass: t == 0, outputs in order
  } else {
#pragma unroll
    for (int r = 0; r < R1; ++r) lds[(t * R1 + r) * CW + c] = v[r];
    lds_passes_but_last<T, N, TH, -1, R1>(lds, tw, t, c);
    constexpr int NSL = LastNS<N, R1>::value;
    lds_pass<T, N, TH, -1, NSL, true>(lds, tw, t, c, store);
  }
}

template <typename T, int N, int TH>
hipError_t launch_fwd_n(const Geometry& g, const double* x, T* spec, const T* gam,
                        const cplx<T>* tw, hipStream_t s) {
  constexpr int CW = Cfg<N, TH>::CW;
  const int nseg = (g.P1 + 2 * CW - 1) / (2 * CW);
  const int64_t nblk = (int64_t)nseg * g.P2 * g.P3;
  hipLaunchKernelGGL((k_time_fwd<T, N, TH>), dim3((unsigned)nblk), dim3(TH), 0, s, x, spec, gam,
                     tw, g.m1, g.m2, g.m3, g.P1, g.P2, g.PS, nseg);
  return hipGetLastError();
}

template <typename T, int N, int TH>
hipError_t launch_inv_n(const Geometry& g, const T* spec, double* z, const T* ginv,
                        const cplx<T>* tw, hipStream_t s) {
  constexpr int CW = Cfg<N, TH>::CW;
  const int nseg = (g.m1 + 2 * CW - 1) / (2 * CW);
  const int64_t nblk = (int64_t)nseg * g.m2 * g.m3;
  hipLaunchKernelGGL((k_time_inv<T, N, TH>), dim3((unsigned)nblk), dim3(TH), 0, s, spec, z,
                     ginv, tw, g.m1, g.m2, g.m3, g.P1, g.P2, g.PS, nseg);
  return hipGetLastError();
}

// 512-thread blocks for n >= 128 once the [n][m] array (FP64) exceeds the
// 256 MiB last-level cache; below that the 256-thread shape is as fast or faster.
template <int N> struct WideTH { static constexpr int value = N >= 128 ? 512 : 256; };
template <int N> bool wide_strips(const Geometry& g) {
  return N >= 128 && (int64_t)N * g.m * 8 > (int64_t(256) << 20);
}

#define AAO_FOR_EACH_N(X) \
  X(2) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024)

template <typename T>
hipError_t dispatch_fwd(const Geometry& g, const double* x, T* spec, const T* gam, const T* tw,
                        hipStream_t s) {
  const cplx<T>* twc = reinterpret_cast<const cplx<T>*>(tw);
  switch (g.n) {
#define CASE(NN) \
  case NN:                                                                          \
    return wide_strips<NN>(g) ? launch_fwd_n<T, NN, WideTH<NN>::value>(g, x, spec, gam, twc, s) \
                              : launch_fwd_n<T, NN, 256>(g, x, spec, gam, twc, s);
    AAO_FOR_EACH_N(CASE)
#undef CASE
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t dispatch_inv(const Geometry& g, const T* spec, double* z, const T* ginv, const T* tw,
                        hipStream_t s) {
  const cplx<T>* twc = reinterpret_cast<const cplx<T>*>(tw);
  switch (g.n) {
#define CASE(NN) \
  case NN:                                                                         \
    return wide_strips<NN>(g) ? launch_inv_n<T, NN, WideTH<NN>::value>(g, spec, z, ginv, twc, s) \
                              : launch_inv_n<T, NN, 256>(g, spec, z, ginv, twc, s);
    AAO_FOR_EACH_N(CASE)
#undef CASE
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_time_fwd_f64(const Geometry& g, const double* x, double* spec,
                               const double* gam, const double* tw, hipStream_t s) {
  return dispatch_fwd<double>(g, x, spec, gam, tw, s);
}
hipError_t launch_time_fwd_f32(const Geometry& g, const double* x, float* spec, const float* gam,
                               const float* tw, hipStream_t s) {
  return dispatch_fwd<float>(g, x, spec, gam, tw, s);
}
hipError_t launch_time_inv_f64(const Geometry& g, const double* spec, double* z,
                               const double* ginv, const double* tw, hipStream_t s) {
  return dispatch_inv<double>(g, spec, z, ginv, tw, s);
}
hipError_t launch_time_inv_f32(const Geometry& g, const float* spec, double* z, const float* ginv,
                               const float* tw, hipStream_t s) {
  return dispatch_inv<float>(g, spec, z, ginv, tw, s);
}

}  // namespace aao
