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
// The FFT is a Stockham autosort sequence of radix-16 (last: smaller) passes
// (radix 8 where radix 16 would spill registers);
// each thread keeps its butterfly's points in registers and the passes
// exchange through one LDS tile of n x CW complex values.  The forward runs its
// first pass on the values it loaded; the inverse stages the half spectrum in
// LDS and its last pass goes straight to HBM.  Both kernels are persistent over
// the column strips (xcd_strips): each block loads the next strip's inputs into
// registers while the LDS passes of the current one run.
//
// Output of Step 1 (input of Step 3) is the split-plane spectrum layout:
//   spec[k][0][i3][i2][i1] = Re, spec[k][1][i3][i2][i1] = Im, planes padded to
//   P1 x P2 x P3; Step 1 writes zeros into every padding position it covers.
#include "common.h"

namespace aao {
namespace {

// TH threads per block: 256, or 512 for long transforms of HBM-resident data
// (wider column strips per block keep more of each DRAM page per request).
template <int N, int TH, int RX> struct Cfg {
  static constexpr int R1 = N < RX ? N : RX;
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
// Results go back to LDS unless FINAL, in which case sink(i0, di, value) gets
// the one at index i0 + di (di a compile-time multiple of NS, i0 per thread).
template <typename T, int N, int TH, int RX, int SIGN, int NS, bool FINAL, typename Sink>
__device__ __forceinline__ void lds_pass(cplx<T>* lds, const cplx<T>* __restrict__ tw, int t,
                                         int c, Sink&& sink) {
  using C = cplx<T>;
  constexpr int TPC = Cfg<N, TH, RX>::TPC, CW = Cfg<N, TH, RX>::CW;
  constexpr int R = (N / NS) < RX ? (N / NS) : RX;
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
      v[q][r] = (r == 0 || NS == 1) ? d : twiddle<T, SIGN>(tw, (r * e) & (N - 1), d);
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
        sink(idxD, r * NS, v[q][r]);
      else
        lds[(idxD + r * NS) * CW + c] = v[q][r];
    }
  }
}

// All passes after the first, writing back to LDS, ending with a barrier.
template <typename T, int N, int TH, int RX, int SIGN, int NS>
__device__ __forceinline__ void lds_passes_all(cplx<T>* lds, const cplx<T>* __restrict__ tw, int t,
                                               int c) {
  if constexpr (NS < N) {
    lds_pass<T, N, TH, RX, SIGN, NS, false>(lds, tw, t, c, [](int, cplx<T>) {});
    constexpr int R = (N / NS) < RX ? (N / NS) : RX;
    lds_passes_all<T, N, TH, RX, SIGN, NS * R>(lds, tw, t, c);
  } else {
    __syncthreads();
  }
}

// Passes after the first except the last (which the caller runs as FINAL).
template <typename T, int N, int TH, int RX, int SIGN, int NS>
__device__ __forceinline__ void lds_passes_but_last(cplx<T>* lds, const cplx<T>* __restrict__ tw,
                                                    int t, int c) {
  constexpr int R = (N / NS) < RX ? (N / NS) : RX;
  if constexpr (NS * R < N) {
    lds_pass<T, N, TH, RX, SIGN, NS, false>(lds, tw, t, c, [](int, cplx<T>) {});
    lds_passes_but_last<T, N, TH, RX, SIGN, NS * R>(lds, tw, t, c);
  }
}

template <int N, int NS, int RX> struct LastNS {
  static constexpr int R = (N / NS) < RX ? (N / NS) : RX;
  static constexpr int value =
      (NS * R >= N) ? NS : LastNS<N, (NS * R >= N ? N : NS * R), RX>::value;
};
template <int N, int RX> struct LastNS<N, N, RX> { static constexpr int value = N; };

// ---------------------------------------------------------------- forward (Step 1)
template <typename T, int N, int TH, int RX>
__global__ __launch_bounds__(TH) __attribute__((amdgpu_waves_per_eu(2))) void k_time_fwd(
    const double* __restrict__ x, T* __restrict__ spec, const T* __restrict__ gam,
    const cplx<T>* __restrict__ tw, int m1, int m2, int m3, int P1, int P2, int64_t PS,
    int nseg, int nstrip) {
  using C = cplx<T>;
  constexpr int R1 = Cfg<N, TH, RX>::R1, TPC = Cfg<N, TH, RX>::TPC, CW = Cfg<N, TH, RX>::CW;
  __shared__ C lds[N * CW];
  __shared__ C twl[N];
  __shared__ T gl[N];
  const int tid = threadIdx.x;
  const int c = tid % CW, t = tid / CW;
  const int64_t m = (int64_t)m1 * m2 * m3;
  for (int j = tid; j < N; j += TH) {
    gl[j] = gam[j];
    twl[j] = tw[j];
  }

  // strip b: column segment sg of spatial row (i2, i3); the two real columns of
  // complex column c are i1a and i1a + CW, so every load and store instruction
  // of a wave covers contiguous addresses
  // The prefetched values stay raw until the next strip starts: a select or
  // conversion right after the load would make the wave wait for it there.
  double ra[R1], rb[R1];
  bool pva = false, pvb = false;   // validity of the prefetched columns
  auto load = [&](int b) {
    const int sg = b % nseg, row = b / nseg, i2 = row % P2, i3 = row / P2;
    const int i1a = sg * 2 * CW + c;
    const bool rowvalid = (i2 < m2) && (i3 < m3);
    pva = rowvalid && i1a < m1;
    pvb = rowvalid && i1a + CW < m1;
    // Loads are unconditional: lanes outside the grid read a clamped in-range
    // point, dropped by the select at use.  Addresses are a per-lane base plus
    // a wave-uniform stride per row, so no per-row 64-bit offset stays live
    // across strips.
    const int64_t rowoff = ((int64_t)min(i3, m3 - 1) * m2 + min(i2, m2 - 1)) * m1 + (int64_t)t * m;
    const double* xa = x + rowoff + min(i1a, m1 - 1);
    const double* xb = x + rowoff + min(i1a + CW, m1 - 1);
    const int64_t step = (int64_t)TPC * m;
#pragma unroll
    for (int r = 0; r < R1; ++r) {
      ra[r] = xa[r * step];
      rb[r] = xb[r * step];
    }
  };

  const StripRange sr = xcd_strips(nstrip);
  if (sr.first < sr.end) load(sr.first);
  __syncthreads();  // gl, twl
  for (int b = sr.first; b < sr.end; b += sr.step) {
    C v[R1];
#pragma unroll
    for (int r = 0; r < R1; ++r) {
      const T gj = gl[t + r * TPC];
      v[r] = {pva ? (T)ra[r] * gj : T(0), pvb ? (T)rb[r] * gj : T(0)};
    }
    if (b + sr.step < sr.end) load(b + sr.step);
    dft<T, R1, +1>(v);
    __syncthreads();  // the previous strip's untangle has read lds
#pragma unroll
    for (int r = 0; r < R1; ++r) lds[(t * R1 + r) * CW + c] = v[r];
    lds_passes_all<T, N, TH, RX, +1, R1>(lds, twl, t, c);

    // untangle: A(k) = (C(k) + conj C(n-k))/2, B(k) = (C(k) - conj C(n-k))/(2i)
    const int sg = b % nseg, row = b / nseg, i2 = row % P2, i3 = row / P2;
    const int i1a = sg * 2 * CW + c, i1b = i1a + CW;
    const bool rowvalid = (i2 < m2) && (i3 < m3);
    const bool va = rowvalid && i1a < m1, vb = rowvalid && i1b < m1;
    const int64_t poff = ((int64_t)i3 * P2 + i2) * P1;
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
}

// ---------------------------------------------------------------- inverse (Step 3)
// Each spectrum value is loaded once: block k <= n/2 gives C(k) = A(k) + i B(k)
// and, through A(n-k) = conj A(k), C(n-k) = conj A(k) + i conj B(k); both are
// staged in LDS, then the Stockham passes run from LDS, the last to HBM.
// No register cap beyond the launch bound: with 256 threads the kernel runs
// one wave per SIMD without spilling, which measures faster than two waves
// with spills (spill reloads share the counter the prefetched loads wait on).
template <typename T, int N, int TH, int RX>
__global__ __launch_bounds__(TH) void k_time_inv(
    const T* __restrict__ spec, double* __restrict__ z, const T* __restrict__ ginv,
    const cplx<T>* __restrict__ tw, int m1, int m2, int m3, int P1, int P2, int64_t PS,
    int nseg, int nstrip) {
  using C = cplx<T>;
  constexpr int TPC = Cfg<N, TH, RX>::TPC, CW = Cfg<N, TH, RX>::CW;
  constexpr int KI = (N / 2) / TPC + 1;  // loads per thread cover k = t + TPC i <= n/2
  __shared__ C lds[N * CW];
  __shared__ C twl[N];
  __shared__ T gl[N];
  const int tid = threadIdx.x;
  const int c = tid % CW, t = tid / CW;
  const int64_t m = (int64_t)m1 * m2 * m3;
  for (int j = tid; j < N; j += TH) {
    gl[j] = ginv[j];
    twl[j] = tw[j];
  }

  // raw prefetched values; selects are applied when the next strip starts
  T ar[KI], ai[KI], br[KI], bi[KI];
  bool pva = false, pvb = false;
  auto load = [&](int b) {
    const int sg = b % nseg, row = b / nseg, i2 = row % m2, i3 = row / m2;
    const int i1a = sg * 2 * CW + c;
    pva = i1a < m1;
    pvb = i1a + CW < m1;
    // unconditional loads from clamped in-range addresses (columns past m1,
    // blocks past n/2); the imaginary planes of blocks 0 and n/2 are read but
    // never used
    const int64_t rowoff = ((int64_t)i3 * P2 + i2) * P1 + (int64_t)t * 2 * PS;
    const T* pa = spec + rowoff + min(i1a, m1 - 1);
    const T* pb = spec + rowoff + min(i1a + CW, m1 - 1);
    const int64_t step = (int64_t)TPC * 2 * PS;
#pragma unroll
    for (int i = 0; i < KI; ++i) {
      // k = t + TPC i <= n/2 always holds except on the last load (t > 0);
      // keeping the other offsets wave-uniform keeps them out of VGPRs
      const int64_t o = (i < KI - 1 || t == 0) ? i * step : 0;
      ar[i] = pa[o];
      ai[i] = pa[o + PS];
      br[i] = pb[o];
      bi[i] = pb[o + PS];
    }
  };

  const StripRange sr = xcd_strips(nstrip);
  if (sr.first < sr.end) load(sr.first);
  for (int b = sr.first; b < sr.end; b += sr.step) {
    __syncthreads();  // the previous strip's last pass has read lds
#pragma unroll
    for (int i = 0; i < KI; ++i) {
      const int k = t + TPC * i;
      if (k <= N / 2) {
        const bool cplxblk = k != 0 && k != N / 2;
        const T a0 = pva ? ar[i] : T(0), b0 = pvb ? br[i] : T(0);
        const T a1 = (pva && cplxblk) ? ai[i] : T(0), b1 = (pvb && cplxblk) ? bi[i] : T(0);
        lds[k * CW + c] = C{a0 - b1, a1 + b0};
        if (cplxblk) lds[(N - k) * CW + c] = C{a0 + b1, b0 - a1};
      }
    }
    if (b + sr.step < sr.end) load(b + sr.step);

    const int sg = b % nseg, row = b / nseg, i2 = row % m2, i3 = row / m2;
    const int i1a = sg * 2 * CW + c;
    const bool va = i1a < m1, vb = i1a + CW < m1;
    double* zb = z + ((int64_t)i3 * m2 + i2) * m1 + i1a;
    auto store = [&](int j0, int dj, C val) {
      const T g = gl[j0 + dj];
      double* zp = zb + (int64_t)j0 * m + dj * m;
      if (va) zp[0] = (double)(val.x * g);
      if (vb) zp[CW] = (double)(val.y * g);
    };
    lds_passes_but_last<T, N, TH, RX, -1, 1>(lds, twl, t, c);
    constexpr int NSL = LastNS<N, 1, RX>::value;
    lds_pass<T, N, TH, RX, -1, NSL, true>(lds, twl, t, c, store);
  }
}

template <typename T, int N, int TH, int RX = 16>
hipError_t launch_fwd_n(const Geometry& g, const double* x, T* spec, const T* gam,
                        const cplx<T>* tw, hipStream_t s) {
  constexpr int CW = Cfg<N, TH, RX>::CW;
  const int nseg = (g.P1 + 2 * CW - 1) / (2 * CW);
  const int64_t ns = (int64_t)nseg * g.P2 * g.P3;
  if (ns > INT32_MAX) return hipErrorInvalidValue;
  static const int resident = persistent_grid(k_time_fwd<T, N, TH, RX>, TH);
  if (resident < 8) return hipErrorInvalidDeviceFunction;
  hipLaunchKernelGGL((k_time_fwd<T, N, TH, RX>), dim3(strip_grid(resident, ns)), dim3(TH), 0, s,
                     x, spec, gam, tw, g.m1, g.m2, g.m3, g.P1, g.P2, g.PS, nseg, (int)ns);
  return hipGetLastError();
}

template <typename T, int N, int TH, int RX = 16>
hipError_t launch_inv_n(const Geometry& g, const T* spec, double* z, const T* ginv,
                        const cplx<T>* tw, hipStream_t s) {
  constexpr int CW = Cfg<N, TH, RX>::CW;
  const int nseg = (g.m1 + 2 * CW - 1) / (2 * CW);
  const int64_t ns = (int64_t)nseg * g.m2 * g.m3;
  if (ns > INT32_MAX) return hipErrorInvalidValue;
  static const int resident = persistent_grid(k_time_inv<T, N, TH, RX>, TH);
  if (resident < 8) return hipErrorInvalidDeviceFunction;
  hipLaunchKernelGGL((k_time_inv<T, N, TH, RX>), dim3(strip_grid(resident, ns)), dim3(TH), 0, s,
                     spec, z, ginv, tw, g.m1, g.m2, g.m3, g.P1, g.P2, g.PS, nseg, (int)ns);
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

// Largest radix of the inverse passes.  The FP64 n = 256 inverse with radix
// 16 needs more than the 256 registers two waves per SIMD leave it and spills
// (54 registers); radix 8 (three passes instead of two) fits in 148 without
// spilling and measured 2.55 ms against 2.78 ms per launch at 127^3 x 256.
// At n = 512 the radix-16 spill is small (5 registers) and radix 16 is faster.
template <typename T, int N> struct InvRadix {
  static constexpr int value = (sizeof(T) == 8 && N == 256) ? 8 : 16;
};

template <typename T>
hipError_t dispatch_inv(const Geometry& g, const T* spec, double* z, const T* ginv, const T* tw,
                        hipStream_t s) {
  const cplx<T>* twc = reinterpret_cast<const cplx<T>*>(tw);
  switch (g.n) {
#define CASE(NN) \
  case NN:                                                                         \
    return wide_strips<NN>(g)                                                          \
               ? launch_inv_n<T, NN, WideTH<NN>::value, InvRadix<T, NN>::value>(          \
                     g, spec, z, ginv, twc, s)                                             \
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
