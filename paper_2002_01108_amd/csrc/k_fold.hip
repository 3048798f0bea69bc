// Folded DST-I mode product on the matrix cores (constant-coefficient Step 2,
// Section 4, eq. (blockdiaginv)).  S_{ij} = sqrt(2/(m+1)) sin((i+1)(j+1) pi/(m+1))
// obeys S_{m-1-r, c} = (-1)^c S_{r, c} (0-based), so with
//   O_r = sum_{c even} S_{r c} x_c,   E_r = sum_{c odd} S_{r c} x_c   (r < h = ceil(m/2))
// the product is y_r = O_r + E_r and y_{m-1-r} = O_r - E_r: two half-size dense
// products (S_oe = S[0:h, 0::2], S_oo = S[0:h, 1::2], zero-padded to Hp x Hp,
// Hp = P/2) instead of one, half the matrix-core work.
//
// Both planes (Re, Im) of a frequency block go through the same block, so the
// S fragments are reused twice and the shifted divide of the last forward
// product (by lambda_k + sum_d tau mu_{i_d}) runs in the epilogue.
//   LEFT  (axis y or z): out[k][pl][o][a][c] = sum_b S[a][b] in[k][pl][o][b][c]
//   RIGHT (axis x):      out[k][pl][rho][a]  = sum_b in[k][pl][rho][b] S[b][a]
// Block tile: FR half-indices r x 64 columns (LEFT) or 64 rows x FR r (RIGHT),
// FR = 64 when P_d/2 allows it (else 32), K slice 8, LDS double buffer, 4 waves
// of 16 columns (rows) each.  Padding positions are written as zero.
#include <type_traits>

#include "common.h"

namespace aao {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mf;
template <> struct Mf<double> {
  typedef d4 V;
  static __device__ __forceinline__ V mfma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <> struct Mf<float> {
  typedef f4 V;
  static __device__ __forceinline__ V mfma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};

constexpr int FBK = 8;     // K slice (half indices t)
constexpr int FC = 64;     // column (LEFT) / row (RIGHT) tile
// LDS row padding: rows of 64 + 16 elements start 128 B (FP64) / 64 B (FP32)
// apart modulo the bank width, so the four k-rows an MFMA operand read touches
// fall on disjoint banks
constexpr int PD = 16;

// Position of a block's tile and its lane in the one-level fold kernels.
struct FoldTile {
  int tid, w, lr, lk, rt, r0, d0, o, k;
  bool real_pair;
  int64_t base0, base1;
};

// Epilogue of the one-level fold (shared by the FP64/FP32 and BF16x3 kernels:
// their accumulators have the same 16x16 layout): y_r = O + E,
// y_{m-1-r} = O - E, the optional complex divide (tax: tau mu along the
// product's axis, in LDS), Q1 scaling, and zero padding.
template <typename T, int NS, bool LEFT, bool DIVIDE, typename V>
__device__ __forceinline__ void fold_epilogue(const V (&acc)[2][2][NS], const FoldTile& tl,
                                              T* __restrict__ out, const FoldArgs& f,
                                              const double* tax, const double* __restrict__ lam,
                                              const double* __restrict__ tmu1,
                                              const double* __restrict__ tmu2,
                                              const double* __restrict__ tmu3) {
  const int tid = tl.tid, w = tl.w, lr = tl.lr, lk = tl.lk, rt = tl.rt;
  const int r0 = tl.r0, d0 = tl.d0, o = tl.o, k = tl.k;
  const bool real_pair = tl.real_pair;
  const int64_t base0 = tl.base0, base1 = tl.base1;
  const int m = f.m, h = (m + 1) / 2;
  T* ob0 = out + base0;
  T* ob1 = out + base1;
  const double lre = DIVIDE ? lam[2 * k] : 0.0, lim = DIVIDE ? lam[2 * k + 1] : 0.0;
  // real pair: lambda_0 and lambda_{n/2} are real
  const double lre1 = (DIVIDE && real_pair) ? lam[2 * f.nk] : 0.0;
  // divisor terms of the two non-product axes: constant per lane (LEFT) or
  // per accumulator row v (RIGHT)
  double cst[4] = {0.0, 0.0, 0.0, 0.0};
  if (DIVIDE) {
    if (LEFT) {
      const int dl = d0 + w * 16 + lr;
      const double c0 = f.axis == 1 ? tmu1[dl] + (tmu3 ? tmu3[o] : 0.0)
                                    : tmu1[dl % f.P1] + tmu2[dl / f.P1];
#pragma unroll
      for (int v = 0; v < 4; ++v) cst[v] = c0;
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int dr = d0 + w * 16 + Mf<T>::row(lk, v);
        cst[v] = tmu2[dr % f.P2] + (tmu3 ? tmu3[dr / f.P2] : 0.0);
      }
    }
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int r, dpos;   // half index and data position (column for LEFT, row for RIGHT)
      if (LEFT) { r = r0 + s * 16 + Mf<T>::row(lk, v); dpos = d0 + w * 16 + lr; }
      else { r = r0 + s * 16 + lr; dpos = d0 + w * 16 + Mf<T>::row(lk, v); }
      if (r >= h) continue;
      // position of the data index in the full grid (for validity and the divide)
      int i1, i2, i3;
      if (LEFT) {
        if (f.axis == 1) { i1 = dpos; i2 = 0; i3 = o; }          // y-mode: column = x, outer = z
        else { i1 = dpos % f.P1; i2 = dpos / f.P1; i3 = 0; }    // z-mode: column = (y, x)
      } else {
        i1 = 0; i2 = dpos % f.P2; i3 = dpos / f.P2;              // x-mode: row = (z, y)
      }
      const bool dvalid = i1 < f.m1 && i2 < f.m2 && i3 < f.m3;
      const T ore = acc[0][0][s][v], ere = acc[0][1][s][v];
      const T oim = acc[1][0][s][v], eim = acc[1][1][s][v];
      const int a_top = r, a_bot = m - 1 - r;
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const int a = half ? a_bot : a_top;
        if (half && a_bot <= a_top) break;
        T vr = half ? ore - ere : ore + ere;
        T vi = half ? oim - eim : oim + eim;
        if (!dvalid) {
          vr = T(0);
          vi = T(0);
        } else if (DIVIDE) {
          const double mu = cst[v] + tax[a];
          if (real_pair) {
            vr = vr / (T)(lre + mu);
            vi = vi / (T)(lre1 + mu);
          } else {
            const T cc = (T)(lre + mu), dd = (T)lim;
            const T inv = T(1) / (cc * cc + dd * dd);
            const T nr = (vr * cc + vi * dd) * inv;
            const T ni = (vi * cc - vr * dd) * inv;
            vr = nr;
            vi = ni;
          }
          if (LEFT && f.ims_r) {
            // Q1 elements: B_k = M (lambda_k I + tau M^{-1} K) in the sine basis
            const T ms = (T)(f.ims_c[dpos] * f.ims_r[a]);
            vr *= ms;
            vi *= ms;
          }
        }
        int64_t off;
        if (LEFT) off = (int64_t)a * f.R + dpos;
        else off = (int64_t)dpos * f.R + a;
        ob0[off] = vr;
        ob1[off] = vi;
      }
    }
  }
  // output indices m .. 2 Hp - 1 along the axis are padding: zero them for this data tile
  if (rt == 0) {
    const int np = 2 * f.Hp - m, cnt = 2 * np * FC;
    for (int e = tid; e < cnt; e += 256) {
      const int pl = e / (np * FC), rem = e % (np * FC);
      int64_t off;
      if (LEFT) off = (int64_t)(m + rem / FC) * f.R + d0 + rem % FC;
      else off = (int64_t)(d0 + rem / np) * f.R + m + rem % np;
      (pl ? ob1 : ob0)[off] = T(0);
    }
  }
}

template <typename T, int FR, bool LEFT, bool DIVIDE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_dst_fold(const T* __restrict__ in, T* __restrict__ out,
                                                  const T* __restrict__ Soe,
                                                  const T* __restrict__ Soo, FoldArgs f,
                                                  const double* __restrict__ lam,
                                                  const double* __restrict__ tmu1,
                                                  const double* __restrict__ tmu2,
                                                  const double* __restrict__ tmu3) {
  using V = typename Mf<T>::V;
  constexpr int NS = FR / 16;            // 16-wide sub-tiles per wave
  constexpr int SPT = 2 * FR * FBK / 256;  // S elements per thread per K slice
  constexpr int STR = FBK / SPT;         // threads per S row
  // LEFT: As = S tiles [mat][t][r], Bs = data [pl][par][t][c]
  // RIGHT: As = data [pl][par][t][row], Bs = S^T tiles [mat][t][r]
  __shared__ T Sd[2][2][2][FBK][FC + PD];   // [buf][pl][par][t][c or row]
  __shared__ T Ss[2][2][FBK][FR + PD];      // [buf][mat][t][r]
  __shared__ double tax[DIVIDE ? 1024 : 1]; // divide: tau mu along the product's axis

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;

  int bid = xcd_remap(blockIdx.x, gridDim.x);
  // tiles: half-index tile fastest (the data tile is reused across it), then data tile, then batch
  const int nrt = f.Hp / FR;
  const int rt = bid % nrt;
  bid /= nrt;
  const int dt = bid % f.ndt;   // LEFT: column tile; RIGHT: row tile
  bid /= f.ndt;
  const int o = bid % f.nout;   // LEFT: outer index; RIGHT: unused (nout = 1)
  const int k = bid / f.nout;
  const int r0 = rt * FR, d0 = dt * FC;
  // plane bases: block k holds (Re, Im) of frequency k; with f.packed, block 0
  // holds the real planes of frequencies 0 and n/2 (both blocks are real when
  // the time data is real) and block k >= 1 frequency k
  const bool real_pair = f.packed && k == 0;
  const int64_t base0 = (int64_t)k * 2 * f.PS + (int64_t)o * f.OS;
  const int64_t base1 = real_pair ? (int64_t)f.nk * 2 * f.PS + (int64_t)o * f.OS : base0 + f.PS;

  // global -> register staging
  T rs[SPT], rd[8];
  // S loads: 2 mats x FR r x FBK t, SPT consecutive t per thread
  const int s_mat = tid >> 7, s_r = (tid & 127) / STR, s_t = ((tid & 127) % STR) * SPT;
  const T* Sm = s_mat ? Soo : Soe;
  // data loads: 2 planes x 2*FBK input indices x FC = 2048, 8 per thread.
  // LEFT: wave w loads plane w/2, parity w%2: lane = column, one row of 64
  // consecutive elements per load.  RIGHT: 2 threads per data row, 8
  // consecutive inputs each.
  const int d_pl = w >> 1, d_par = w & 1;
  int d_a, d_c;   // RIGHT: data row (0..63) and first of 8 inputs
  if (LEFT) { d_a = 0; d_c = 0; }
  else { d_a = (tid & 127) >> 1; d_c = (tid & 1) * 8; }

  auto fetch = [&](int t0) {
#pragma unroll
    for (int e = 0; e < SPT; ++e) rs[e] = Sm[(int64_t)(r0 + s_r) * f.Hp + t0 + s_t + e];
    const T* src = in + (d_pl ? base1 : base0);
    if (LEFT) {
      const T* p = src + (int64_t)(2 * t0 + d_par) * f.R + d0 + lane;
#pragma unroll
      for (int e = 0; e < 8; ++e) rd[e] = p[(int64_t)(2 * e) * f.R];
    } else {
      const T* p = src + (int64_t)(d0 + d_a) * f.R + 2 * t0 + d_c;
#pragma unroll
      for (int e = 0; e < 8; ++e) rd[e] = p[e];
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int e = 0; e < SPT; ++e) Ss[buf][s_mat][s_t + e][s_r] = rs[e];
    if (LEFT) {
      // input row 2(t0+e)+par -> (par, e)
#pragma unroll
      for (int e = 0; e < 8; ++e) Sd[buf][d_pl][d_par][e][lane] = rd[e];
    } else {
      // input column 2t+par of data row d_a
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int cidx = d_c + e;
        Sd[buf][d_pl][cidx & 1][cidx >> 1][d_a] = rd[e];
      }
    }
  };

  V acc[2][2][NS];   // [plane][O/E][sub-tile]
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int s = 0; s < NS; ++s) acc[a][b][s] = V{0, 0, 0, 0};

  // divide: stage the axis table in LDS (read by the epilogue after the barriers)
  if (DIVIDE) {
    const double* ax_tab = LEFT ? (f.axis == 1 ? tmu2 : tmu3) : tmu1;
    for (int i = tid; i < 2 * f.Hp; i += 256) tax[i] = ax_tab[i];
  }
  fetch(0);
  stash(0);
  __syncthreads();
  const int nk = f.Hp / FBK;
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) fetch((kt + 1) * FBK);
#pragma unroll
    for (int ks = 0; ks < FBK / 4; ++ks) {
      const int kk = ks * 4 + lk;
      if (LEFT) {
        T a[2][NS], b[2][2];   // a[mat][i], b[pl][par]
#pragma unroll
        for (int mat = 0; mat < 2; ++mat)
#pragma unroll
          for (int i = 0; i < NS; ++i) a[mat][i] = Ss[buf][mat][kk][i * 16 + lr];
#pragma unroll
        for (int pl = 0; pl < 2; ++pl)
#pragma unroll
          for (int par = 0; par < 2; ++par) b[pl][par] = Sd[buf][pl][par][kk][w * 16 + lr];
#pragma unroll
        for (int pl = 0; pl < 2; ++pl)
#pragma unroll
          for (int oe = 0; oe < 2; ++oe)
#pragma unroll
            for (int i = 0; i < NS; ++i)
              acc[pl][oe][i] = Mf<T>::mfma(a[oe][i], b[pl][oe], acc[pl][oe][i]);
      } else {
        T a[2][2], b[2][NS];   // a[pl][par], b[mat][j]
#pragma unroll
        for (int pl = 0; pl < 2; ++pl)
#pragma unroll
          for (int par = 0; par < 2; ++par) a[pl][par] = Sd[buf][pl][par][kk][w * 16 + lr];
#pragma unroll
        for (int mat = 0; mat < 2; ++mat)
#pragma unroll
          for (int j = 0; j < NS; ++j) b[mat][j] = Ss[buf][mat][kk][j * 16 + lr];
#pragma unroll
        for (int pl = 0; pl < 2; ++pl)
#pragma unroll
          for (int oe = 0; oe < 2; ++oe)
#pragma unroll
            for (int j = 0; j < NS; ++j)
              acc[pl][oe][j] = Mf<T>::mfma(a[pl][oe], b[oe][j], acc[pl][oe][j]);
      }
    }
    if (kt + 1 < nk) stash(buf ^ 1);
    __syncthreads();
  }

  fold_epilogue<T, NS, LEFT, DIVIDE>(acc, FoldTile{tid, w, lr, lk, rt, r0, d0, o, k, real_pair, base0, base1},
                                     out, f, tax, lam, tmu1, tmu2, tmu3);
}

template <typename T, int FR>
hipError_t launch_fold_fr(const T* in, T* out, const T* Soe, const T* Soo, const FoldArgs& f,
                          bool left, const double* lam, const double* tmu1, const double* tmu2,
                          const double* tmu3, hipStream_t s) {
  const int64_t nblk = (int64_t)(f.Hp / FR) * f.ndt * f.nout * f.nk;
  if (nblk > 0x7fffffff || nblk < 1) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)nblk), blk(256);
  const bool div = lam != nullptr;
  if (left) {
    if (div)
      hipLaunchKernelGGL((k_dst_fold<T, FR, true, true>), grid, blk, 0, s, in, out, Soe, Soo, f,
                         lam, tmu1, tmu2, tmu3);
    else
      hipLaunchKernelGGL((k_dst_fold<T, FR, true, false>), grid, blk, 0, s, in, out, Soe, Soo, f,
                         lam, tmu1, tmu2, tmu3);
  } else {
    if (div)
      hipLaunchKernelGGL((k_dst_fold<T, FR, false, true>), grid, blk, 0, s, in, out, Soe, Soo, f,
                         lam, tmu1, tmu2, tmu3);
    else
      hipLaunchKernelGGL((k_dst_fold<T, FR, false, false>), grid, blk, 0, s, in, out, Soe, Soo,
                         f, lam, tmu1, tmu2, tmu3);
  }
  return hipGetLastError();
}


// ---------------------------------------------------------------- BF16x3 fold
// The one-level fold with BF16 hi/lo splits on v_mfma_f32_16x16x32_bf16: the
// FP32 data are split while staged (hi = rne(x), lo = rne(x - hi)), the folded
// tables once on the host, and every product accumulates lo*hi + hi*lo + hi*hi
// in FP32.  Three BF16 products cost 3/16 of one FP32 matrix-core product, so
// the pass is bound by HBM even at P_d = 512.  Both LDS operands keep t
// contiguous (a fragment is 8 consecutive t of one row or column: one 16-byte
// read), K slices of 32 half indices, one LDS buffer with the next slice
// prefetched into registers (two buffers would not leave room for two blocks
// per CU).  Rows of 32 + 8 elements (80 bytes): the 16-byte accesses of 16
// consecutive rows cover distinct banks.  Tiles, planes and epilogue as
// k_dst_fold.
typedef __bf16 fbf16x8 __attribute__((ext_vector_type(8)));
typedef short fs8v __attribute__((ext_vector_type(8)));
typedef unsigned short fu16;

typedef __bf16 fbf16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t fu32x4 __attribute__((ext_vector_type(4)));
// hi = rne(x), lo = rne(x - hi) of two values, as packed pairs (the
// conversions are v_cvt_pk_bf16_f32: round to nearest even)
__device__ __forceinline__ void fold_split2(float a, float b, uint32_t& hi, uint32_t& lo) {
  const fbf16x2 h = {(__bf16)a, (__bf16)b};
  hi = __builtin_bit_cast(uint32_t, h);
  const fbf16x2 l = {(__bf16)(a - __uint_as_float(hi << 16)),
                     (__bf16)(b - __uint_as_float(hi & 0xFFFF0000u))};
  lo = __builtin_bit_cast(uint32_t, l);
}

constexpr int XK3 = 32, XR3 = XK3 + 8;   // K slice and LDS row length (bf16 elements)

template <int FR, bool LEFT, bool DIVIDE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_dst_fold_bf3(
    const float* __restrict__ in, float* __restrict__ out, const fu16* __restrict__ Shi_oe,
    const fu16* __restrict__ Slo_oe, const fu16* __restrict__ Shi_oo,
    const fu16* __restrict__ Slo_oo, FoldArgs f, const double* __restrict__ lam,
    const double* __restrict__ tmu1, const double* __restrict__ tmu2,
    const double* __restrict__ tmu3) {
  constexpr int NS = FR / 16;               // 16-wide sub-tiles per wave
  constexpr int SPT = 2 * FR * XK3 / 256;   // table elements per thread and slice (16 or 8)
  constexpr int SQ = SPT / 8;               // 16-byte words of them
  // tables [buffer][hi/lo][O/E][r][t]
  __shared__ __attribute__((aligned(16))) fu16 S3[2][2][2][FR][XR3];
  __shared__ double tax[DIVIDE ? 1024 : 1];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;

  int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int nrt = f.Hp / FR;
  const int rt = bid % nrt;
  bid /= nrt;
  const int dt = bid % f.ndt;
  bid /= f.ndt;
  const int o = bid % f.nout;
  const int k = bid / f.nout;
  const int r0 = rt * FR, d0 = dt * FC;
  const bool real_pair = f.packed && k == 0;
  const int64_t base0 = (int64_t)k * 2 * f.PS + (int64_t)o * f.OS;
  const int64_t base1 = real_pair ? (int64_t)f.nk * 2 * f.PS + (int64_t)o * f.OS : base0 + f.PS;

  // tables: thread -> (O/E, row, SPT consecutive t)
  const int s_mat = tid >> 7;
  const int s_r = (tid & 127) / (XK3 / SPT), s_t = ((tid & 127) % (XK3 / SPT)) * SPT;
  const fu32x4* Sh = reinterpret_cast<const fu32x4*>(s_mat ? Shi_oo : Shi_oe);
  const fu32x4* Sl = reinterpret_cast<const fu32x4*>(s_mat ? Slo_oo : Slo_oe);
  // data: lane (lr, lk) of wave w reads its own operand fragments, the 8 half
  // indices t = t0 + 8 lk + j (j < 8) of both parities and planes at data
  // position d0 + 16 w + lr (LEFT: a column; RIGHT: a row)
  const int dpos = d0 + w * 16 + lr;
  const float* src0 = in + base0;
  const float* src1 = in + base1;

  struct Stage {
    fu32x4 sh[SQ], sl[SQ];
    float d[2][2][8];   // [plane][parity][j]
  };
  auto fetch = [&](int t0, Stage& g) {
    const int64_t so = ((int64_t)(r0 + s_r) * f.Hp + t0 + s_t) / 8;
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
      g.sh[q] = Sh[so + q];
      g.sl[q] = Sl[so + q];
    }
    const int i0 = 2 * (t0 + 8 * lk);   // first input index of the lane
#pragma unroll
    for (int pl = 0; pl < 2; ++pl) {
      const float* src = pl ? src1 : src0;
      if (LEFT) {
        // 16 consecutive input rows of one column, parities interleaved
        const float* p = src + (int64_t)i0 * f.R + dpos;
#pragma unroll
        for (int e = 0; e < 16; ++e) g.d[pl][e & 1][e >> 1] = p[(int64_t)e * f.R];
      } else {
        // 16 consecutive inputs of one data row: four 16-byte loads
        const float4* p = reinterpret_cast<const float4*>(src + (int64_t)dpos * f.R + i0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float4 v = p[q];
          g.d[pl][0][2 * q] = v.x;
          g.d[pl][1][2 * q] = v.y;
          g.d[pl][0][2 * q + 1] = v.z;
          g.d[pl][1][2 * q + 1] = v.w;
        }
      }
    }
  };
  auto stash = [&](int buf, const Stage& g) {
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
      *reinterpret_cast<fu32x4*>(&S3[buf][0][s_mat][s_r][s_t + 8 * q]) = g.sh[q];
      *reinterpret_cast<fu32x4*>(&S3[buf][1][s_mat][s_r][s_t + 8 * q]) = g.sl[q];
    }
  };
  auto frag = [](const fu16* p) {
    return __builtin_bit_cast(fbf16x8, *reinterpret_cast<const fs8v*>(p));
  };
  auto tofrag = [](const uint32_t (&u)[4]) {
    return __builtin_bit_cast(fbf16x8, fu32x4{u[0], u[1], u[2], u[3]});
  };

  f4 acc[2][2][NS];   // [plane][O/E][sub-tile]
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int s = 0; s < NS; ++s) acc[a][b][s] = f4{0, 0, 0, 0};

  // one K slice: the data fragments split in registers, the table fragments
  // from LDS buffer `buf`; oe is a constant so that the accumulators stay in
  // registers
  auto product = [&](auto oe_c, int buf, const fbf16x8 (&dh)[2], const fbf16x8 (&dl)[2]) {
    constexpr int oe = decltype(oe_c)::value;
    const int kc = lk * 8;
    fbf16x8 th[NS], tl[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      th[i] = frag(&S3[buf][0][oe][i * 16 + lr][kc]);
      tl[i] = frag(&S3[buf][1][oe][i * 16 + lr][kc]);
    }
#pragma unroll
    for (int pl = 0; pl < 2; ++pl)
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        f4 c = acc[pl][oe][i];
        if (LEFT) {   // table rows x data columns
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(tl[i], dh[pl], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(th[i], dl[pl], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(th[i], dh[pl], c, 0, 0, 0);
        } else {      // data rows x table rows (S^T)
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dl[pl], th[i], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dh[pl], tl[i], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dh[pl], th[i], c, 0, 0, 0);
        }
        acc[pl][oe][i] = c;
      }
  };
  auto compute = [&](int buf, const Stage& g) {
    // parity par multiplies the O (par 0) or E (par 1) table
    fbf16x8 dh[2][2], dl[2][2];   // [parity][plane]
#pragma unroll
    for (int pl = 0; pl < 2; ++pl)
#pragma unroll
      for (int par = 0; par < 2; ++par) {
        uint32_t h[4], l[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
          fold_split2(g.d[pl][par][2 * e], g.d[pl][par][2 * e + 1], h[e], l[e]);
        dh[par][pl] = tofrag(h);
        dl[par][pl] = tofrag(l);
      }
    product(std::integral_constant<int, 0>{}, buf, dh[0], dl[0]);
    product(std::integral_constant<int, 1>{}, buf, dh[1], dl[1]);
  };

  if (DIVIDE) {
    const double* ax_tab = LEFT ? (f.axis == 1 ? tmu2 : tmu3) : tmu1;
    for (int i = tid; i < 2 * f.Hp; i += 256) tax[i] = ax_tab[i];
  }
  const int nk = f.Hp / XK3;
  // tables double-buffered in LDS (one barrier per slice); the next slice's
  // tables and data are loaded into registers while this one computes
  Stage cur, nxt;
  fetch(0, cur);
  stash(0, cur);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) fetch((kt + 1) * XK3, nxt);
    compute(buf, cur);
    if (kt + 1 < nk) {
      stash(buf ^ 1, nxt);
      cur = nxt;
    }
    __syncthreads();
  }
  fold_epilogue<float, NS, LEFT, DIVIDE>(
      acc, FoldTile{tid, w, lr, lk, rt, r0, d0, o, k, real_pair, base0, base1}, out, f, tax, lam,
      tmu1, tmu2, tmu3);
}

template <int FR>
hipError_t launch_fold_bf3_fr(const float* in, float* out, const fu16* const* T, const FoldArgs& f,
                              bool left, const double* lam, const double* tmu1,
                              const double* tmu2, const double* tmu3, hipStream_t s) {
  const int64_t nblk = (int64_t)(f.Hp / FR) * f.ndt * f.nout * f.nk;
  if (nblk > 0x7fffffff || nblk < 1) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)nblk), blk(256);
#define AAO_BF3(L, D)                                                                        \
  hipLaunchKernelGGL((k_dst_fold_bf3<FR, L, D>), grid, blk, 0, s, in, out, T[0], T[1], T[2], \
                     T[3], f, lam, tmu1, tmu2, tmu3)
  if (left) {
    if (lam) AAO_BF3(true, true);
    else AAO_BF3(true, false);
  } else {
    if (lam) AAO_BF3(false, true);
    else AAO_BF3(false, false);
  }
#undef AAO_BF3
  return hipGetLastError();
}

// ---------------------------------------------------------------- two-level fold (odd m)
// For odd m (h = (m+1)/2) the halves fold once more.  With a the even (b = 0)
// or odd (b = 1) inputs x_{2t+b}, the mirror t' = h-1-t (b = 0) / h-2-t
// (b = 1) satisfies S_{r, 2t'+b} = (-1)^r S_{r, 2t+b}, so with
//   u^+-_t = x_{2t} +- x_{2t'},  v^+-_t = x_{2t+1} +- x_{2t'+1}  (t < t'; the
//   middle t = t' keeps x alone in the + combination)
// the even rows r = 2q use the + combinations and the odd rows r = 2q+1 the -
// combinations: O_r = A^{+-}[q] . u^{+-},  E_r = B^{+-}[q] . v^{+-}, four
// quarter-size products (tables [4][Hq][Hq], Hq = P/4: A+, A-, B+, B-) in
// place of the two half-size ones, then y_r = O_r + E_r, y_{m-1-r} = O_r - E_r
// as before.  Block tile: FQ quarter indices (2 FQ rows r) x 64 columns, FQ = 32
// (FP64) or 64 (FP32 with Hq a multiple of 64: half the blocks re-read a data
// tile); the four +- combinations of a K slice are formed in registers and
// staged in one LDS buffer (register prefetch of the next slice).
template <typename T, bool LEFT, bool DIVIDE, int FQ>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_dst_fold2(
    const T* __restrict__ in, T* __restrict__ out, const T* __restrict__ tabs, FoldArgs f,
    const double* __restrict__ lam, const double* __restrict__ tmu1,
    const double* __restrict__ tmu2, const double* __restrict__ tmu3) {
  using V = typename Mf<T>::V;
  constexpr int NS = FQ / 16;
  // RIGHT stores its slice transposed (16 lanes along a row write 16 different
  // LDS rows); one extra element of padding spreads those rows over the banks
  constexpr int PDS = LEFT ? PD : PD + 1;
  __shared__ T Sd[2][2][2][FBK][FC + PDS];   // [pl][par][sign][t][c or row]
  __shared__ T Ts[4][FBK][FQ + PD];         // [table][t][q]
  __shared__ double tax[DIVIDE ? 1024 : 1];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int Hq = f.Hp / 2, h = (f.m + 1) / 2;

  int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int nqt = Hq / FQ;
  const int qt = bid % nqt;
  bid /= nqt;
  const int dt = bid % f.ndt;
  bid /= f.ndt;
  const int o = bid % f.nout;
  const int k = bid / f.nout;
  const int q0 = qt * FQ, d0 = dt * FC;
  const bool real_pair = f.packed && k == 0;
  const int64_t base0 = (int64_t)k * 2 * f.PS + (int64_t)o * f.OS;
  const int64_t base1 = real_pair ? (int64_t)f.nk * 2 * f.PS + (int64_t)o * f.OS : base0 + f.PS;

  // loads: LEFT: wave w = plane w/2, parity w%2, lane = column, e = t offset.
  // RIGHT: 16 lanes along a data row take the slice's 16 inputs 2 t0 .. 2 t0 + 15
  // (and the 16 mirrored ones, contiguous in reverse), 4 rows per wave; load e
  // covers (plane, row) = g + 16 e.
  const int d_pl = w >> 1;
  const int r_c = tid & 15, r_g = tid >> 4;
  // table staging: 64 threads per table, TPQ of them per quarter index, TE
  // consecutive t each
  constexpr int TPQ = 64 / FQ, TE = FBK / TPQ;
  T xa[8], xb[8], rt_[TE];
  const int t_tab = tid >> 6, t_q = (tid & 63) / TPQ, t_t = ((tid & 63) % TPQ) * TE;

  auto mirror = [&](int t, int par) { return par ? h - 2 - t : h - 1 - t; };
  auto fetch = [&](int t0) {
#pragma unroll
    for (int e = 0; e < TE; ++e)
      rt_[e] = tabs[((int64_t)t_tab * Hq + q0 + t_q) * Hq + t0 + t_t + e];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      int t, par, pl;
      int64_t pa, pb;
      if (LEFT) {
        pl = d_pl;
        par = w & 1;
        t = t0 + e;
        pa = (int64_t)(2 * t + par) * f.R + d0 + lane;
      } else {
        const int idx = r_g + 16 * e;
        pl = idx >> 6;
        par = r_c & 1;
        t = t0 + (r_c >> 1);
        pa = (int64_t)(d0 + (idx & 63)) * f.R + 2 * t0 + r_c;
      }
      // the mirror input exists only for a proper pair (mirror > t); the
      // clamped index keeps the address in range either way
      const int mir = mirror(t, par);
      const int mc = mir > t ? mir : t;
      if (LEFT) pb = (int64_t)(2 * mc + par) * f.R + d0 + lane;
      else pb = (int64_t)(d0 + ((r_g + 16 * e) & 63)) * f.R + 2 * mc + par;
      const T* src = in + (pl ? base1 : base0);
      xa[e] = src[pa];
      xb[e] = mir > t ? src[pb] : T(0);
    }
  };

  V acc[4][2][NS];   // [table][plane][sub-tile]
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < NS; ++c) acc[a][b][c] = V{0, 0, 0, 0};

  if (DIVIDE) {
    const double* ax_tab = LEFT ? (f.axis == 1 ? tmu2 : tmu3) : tmu1;
    for (int i = tid; i < 2 * f.Hp; i += 256) tax[i] = ax_tab[i];
  }
  const int nk = Hq / FBK;
  fetch(0);
  for (int kt = 0; kt < nk; ++kt) {
    const int t0 = kt * FBK;
    __syncthreads();   // every wave is done reading the previous slice
    // combine: + and - of each pair; the middle keeps x alone in +, beyond-
    // the-pairs indices contribute zero (their table columns are zero too)
#pragma unroll
    for (int e = 0; e < TE; ++e) Ts[t_tab][t_t + e][t_q] = rt_[e];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      int lt, par, pl, pos;
      if (LEFT) { par = w & 1; lt = e; pl = d_pl; pos = lane; }
      else {
        const int idx = r_g + 16 * e;
        par = r_c & 1; lt = r_c >> 1; pl = idx >> 6; pos = idx & 63;
      }
      const int t = t0 + lt, mir = mirror(t, par);
      const T a = xa[e], b = xb[e];
      Sd[pl][par][0][lt][pos] = mir >= t ? a + b : T(0);
      Sd[pl][par][1][lt][pos] = mir > t ? a - b : T(0);
    }
    __syncthreads();
    if (kt + 1 < nk) fetch(t0 + FBK);
#pragma unroll
    for (int ks = 0; ks < FBK / 4; ++ks) {
      const int kk = ks * 4 + lk;
      if (LEFT) {
        T a[4][NS], b[2][2][2];   // a[table][i], b[pl][par][sign]
#pragma unroll
        for (int tb = 0; tb < 4; ++tb)
#pragma unroll
          for (int i = 0; i < NS; ++i) a[tb][i] = Ts[tb][kk][i * 16 + lr];
#pragma unroll
        for (int pl = 0; pl < 2; ++pl)
#pragma unroll
          for (int par = 0; par < 2; ++par)
#pragma unroll
            for (int sg = 0; sg < 2; ++sg) b[pl][par][sg] = Sd[pl][par][sg][kk][w * 16 + lr];
#pragma unroll
        for (int tb = 0; tb < 4; ++tb)
#pragma unroll
          for (int pl = 0; pl < 2; ++pl)
#pragma unroll
            for (int i = 0; i < NS; ++i)
              acc[tb][pl][i] = Mf<T>::mfma(a[tb][i], b[pl][tb >> 1][tb & 1], acc[tb][pl][i]);
      } else {
        T a[2][2][2], b[4][NS];   // a[pl][par][sign], b[table][j]
#pragma unroll
        for (int pl = 0; pl < 2; ++pl)
#pragma unroll
          for (int par = 0; par < 2; ++par)
#pragma unroll
            for (int sg = 0; sg < 2; ++sg) a[pl][par][sg] = Sd[pl][par][sg][kk][w * 16 + lr];
#pragma unroll
        for (int tb = 0; tb < 4; ++tb)
#pragma unroll
          for (int j = 0; j < NS; ++j) b[tb][j] = Ts[tb][kk][j * 16 + lr];
#pragma unroll
        for (int tb = 0; tb < 4; ++tb)
#pragma unroll
          for (int pl = 0; pl < 2; ++pl)
#pragma unroll
            for (int j = 0; j < NS; ++j)
              acc[tb][pl][j] = Mf<T>::mfma(a[pl][tb >> 1][tb & 1], b[tb][j], acc[tb][pl][j]);
      }
    }
  }

  // epilogue: row r = 2q + s2 takes tables s2 (O) and 2 + s2 (E);
  // y_r = O + E, y_{m-1-r} = O - E, optional divide, zero padding
  const int m = f.m;
  T* ob0 = out + base0;
  T* ob1 = out + base1;
  const double lre = DIVIDE ? lam[2 * k] : 0.0, lim = DIVIDE ? lam[2 * k + 1] : 0.0;
  const double lre1 = (DIVIDE && real_pair) ? lam[2 * f.nk] : 0.0;
  double cst[4] = {0.0, 0.0, 0.0, 0.0};
  if (DIVIDE) {
    if (LEFT) {
      const int dl = d0 + w * 16 + lr;
      const double c0 = f.axis == 1 ? tmu1[dl] + (tmu3 ? tmu3[o] : 0.0)
                                    : tmu1[dl % f.P1] + tmu2[dl / f.P1];
#pragma unroll
      for (int v = 0; v < 4; ++v) cst[v] = c0;
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int dr = d0 + w * 16 + Mf<T>::row(lk, v);
        cst[v] = tmu2[dr % f.P2] + (tmu3 ? tmu3[dr / f.P2] : 0.0);
      }
    }
  }
#pragma unroll
  for (int sub = 0; sub < NS; ++sub) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int q, dpos;
      if (LEFT) { q = q0 + sub * 16 + Mf<T>::row(lk, v); dpos = d0 + w * 16 + lr; }
      else { q = q0 + sub * 16 + lr; dpos = d0 + w * 16 + Mf<T>::row(lk, v); }
      int i1, i2, i3;
      if (LEFT) {
        if (f.axis == 1) { i1 = dpos; i2 = 0; i3 = o; }
        else { i1 = dpos % f.P1; i2 = dpos / f.P1; i3 = 0; }
      } else {
        i1 = 0; i2 = dpos % f.P2; i3 = dpos / f.P2;
      }
      const bool dvalid = i1 < f.m1 && i2 < f.m2 && i3 < f.m3;
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        const int r = 2 * q + s2;
        if (r >= h) continue;
        const T ore = acc[s2][0][sub][v], ere = acc[2 + s2][0][sub][v];
        const T oim = acc[s2][1][sub][v], eim = acc[2 + s2][1][sub][v];
        const int a_top = r, a_bot = m - 1 - r;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          const int a = half ? a_bot : a_top;
          if (half && a_bot <= a_top) break;
          T vr = half ? ore - ere : ore + ere;
          T vi = half ? oim - eim : oim + eim;
          if (!dvalid) {
            vr = T(0);
            vi = T(0);
          } else if (DIVIDE) {
            const double mu = cst[v] + tax[a];
            if (real_pair) {
              vr = vr / (T)(lre + mu);
              vi = vi / (T)(lre1 + mu);
            } else {
              const T cc = (T)(lre + mu), dd = (T)lim;
              const T inv = T(1) / (cc * cc + dd * dd);
              const T nr = (vr * cc + vi * dd) * inv;
              const T ni = (vi * cc - vr * dd) * inv;
              vr = nr;
              vi = ni;
            }
            if (LEFT && f.ims_r) {
              // Q1 elements: B_k = M (lambda_k I + tau M^{-1} K) in the sine basis
              const T ms = (T)(f.ims_c[dpos] * f.ims_r[a]);
              vr *= ms;
              vi *= ms;
            }
          }
          int64_t off;
          if (LEFT) off = (int64_t)a * f.R + dpos;
          else off = (int64_t)dpos * f.R + a;
          ob0[off] = vr;
          ob1[off] = vi;
        }
      }
    }
  }
  if (qt == 0) {
    const int np = 2 * f.Hp - m, cnt = 2 * np * FC;
    for (int e = tid; e < cnt; e += 256) {
      const int pl = e / (np * FC), rem = e % (np * FC);
      int64_t off;
      if (LEFT) off = (int64_t)(m + rem / FC) * f.R + d0 + rem % FC;
      else off = (int64_t)(d0 + rem / np) * f.R + m + rem % np;
      (pl ? ob1 : ob0)[off] = T(0);
    }
  }
}

template <typename T, int FQ>
hipError_t launch_fold2_fq(const T* in, T* out, const T* tabs, const FoldArgs& f, bool left,
                           const double* lam, const double* tmu1, const double* tmu2,
                           const double* tmu3, hipStream_t s) {
  const int64_t nblk = (int64_t)(f.Hp / 2 / FQ) * f.ndt * f.nout * f.nk;
  if (nblk > 0x7fffffff || nblk < 1) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)nblk), blk(256);
  const bool div = lam != nullptr;
  if (left) {
    if (div)
      hipLaunchKernelGGL((k_dst_fold2<T, true, true, FQ>), grid, blk, 0, s, in, out, tabs, f, lam,
                         tmu1, tmu2, tmu3);
    else
      hipLaunchKernelGGL((k_dst_fold2<T, true, false, FQ>), grid, blk, 0, s, in, out, tabs, f,
                         lam, tmu1, tmu2, tmu3);
  } else {
    if (div)
      hipLaunchKernelGGL((k_dst_fold2<T, false, true, FQ>), grid, blk, 0, s, in, out, tabs, f,
                         lam, tmu1, tmu2, tmu3);
    else
      hipLaunchKernelGGL((k_dst_fold2<T, false, false, FQ>), grid, blk, 0, s, in, out, tabs, f,
                         lam, tmu1, tmu2, tmu3);
  }
  return hipGetLastError();
}

// FP32 takes 64 quarter indices per block where Hq allows it (196-217 VGPRs,
// no spills): at 511^2 x 512 the products take 517-582 us against 571-595 us
// with 32 (FP64 with 64 would not fit the registers)
constexpr int FQ32 = 64;
template <typename T>
hipError_t launch_fold2(const T* in, T* out, const T* tabs, const FoldArgs& f, bool left,
                        const double* lam, const double* tmu1, const double* tmu2,
                        const double* tmu3, hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    if ((f.Hp / 2) % FQ32 == 0)
      return launch_fold2_fq<T, FQ32>(in, out, tabs, f, left, lam, tmu1, tmu2, tmu3, s);
  }
  return launch_fold2_fq<T, 32>(in, out, tabs, f, left, lam, tmu1, tmu2, tmu3, s);
}


// ---------------------------------------------------------------- fused y-fwd, divide, y-inv
// Along the axis of the shifted divide (y in 2D, z in 3D) the forward product,
// the divide and the inverse product run in one kernel (FP64 or FP32) with odd m and
// P = 4 HQ (two-level fold).  A block owns 16 columns (x, or the flattened
// (y, x) for z) of one plane pair: it stages the whole column tile in LDS, each
// wave forms the forward quarter products for 16 quarter indices q, and the
// epilogue of the forward product already yields the inverse product's inputs:
// the rows 2q and m-1-2q (even pair) and 2q+1 and m-2-2q (odd pair) come out of
// the same accumulators, so after the divide u+- = y_2q +- y_(m-1-2q) and
// v+- = y_(2q+1) +- y_(m-2-2q) are formed in registers and stored to LDS in
// place of the column tile.  The inverse product then reads them directly.
// Tables are the same quarter tables, transposed ([table][t][q]) so that lanes
// read consecutive q.
constexpr int FCF = 16;

template <typename T, int HQ>
__global__ __launch_bounds__(64 * (HQ / 16)) __attribute__((amdgpu_waves_per_eu(2))) void k_dst_fold2_fused(
    const T* in, T* out, const T* __restrict__ tt,
    FoldArgs f, const double* __restrict__ lam, const double* __restrict__ tmu1,
    const double* __restrict__ tmu2, const double* __restrict__ tmu3) {
  using V = typename Mf<T>::V;
  using T2 = std::conditional_t<sizeof(T) == 8, double2, float2>;
  constexpr int P = 4 * HQ, NT = 64 * (HQ / 16);
  // the operands of one quarter-product pass, Cc[pl][combo][t][c]: combo
  // 2 par + sign holds x_{2t+par} + x_{2t'+par} (sign 0) or - (sign 1); first
  // the forward product's inputs, then the inverse product's
  __shared__ T Cc[2][4][HQ][FCF];
  __shared__ double tax[P];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int m = f.m, h = (m + 1) / 2;

  int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int dt = bid % f.ndt;
  bid /= f.ndt;
  const int o = bid % f.nout;
  const int k = bid / f.nout;
  const int d0 = dt * FCF, q0 = w * 16;
  const bool real_pair = f.packed && k == 0;
  const int64_t base0 = (int64_t)k * 2 * f.PS + (int64_t)o * f.OS;
  const int64_t base1 = real_pair ? (int64_t)f.nk * 2 * f.PS + (int64_t)o * f.OS : base0 + f.PS;

  // Stage the forward product's operands: for quarter index t and parity par
  // the rows 2t+par and 2t'+par (16 contiguous columns each, two per thread
  // and load) combine into the + and - operands once here, so the product
  // loop only reads LDS.  All loads of a thread are issued before the first
  // LDS store so that their latencies overlap.
  auto mirror = [&](int t, int par) { return par ? h - 2 - t : h - 1 - t; };
  constexpr int NST = 2 * 2 * HQ * (FCF / 2) / NT;   // (pl, par, t, column pair) per thread
  T2 xa[NST], xb[NST];
#pragma unroll
  for (int i = 0; i < NST; ++i) {
    const int e = tid + i * NT, c2 = e % (FCF / 2), r = e / (FCF / 2);
    const int t = r % HQ, par = (r / HQ) & 1, pl = r / (2 * HQ);
    const int mir = mirror(t, par), mc = mir > t ? mir : t;   // in range either way
    const T* src = in + (pl ? base1 : base0) + d0 + 2 * c2;
    xa[i] = *reinterpret_cast<const T2*>(src + (int64_t)(2 * t + par) * f.R);
    xb[i] = *reinterpret_cast<const T2*>(src + (int64_t)(2 * mc + par) * f.R);
  }
#pragma unroll
  for (int i = 0; i < NST; ++i) {
    const int e = tid + i * NT, c2 = e % (FCF / 2), r = e / (FCF / 2);
    const int t = r % HQ, par = (r / HQ) & 1, pl = r / (2 * HQ);
    const int mir = mirror(t, par);
    // a proper pair gives + and -; the middle (t' = t) keeps x alone in +;
    // beyond the pairs both are zero (those rows are another t's mirrors)
    const bool pair = mir > t, mid = mir == t;
    Cc[pl][2 * par][t][2 * c2] = pair ? xa[i].x + xb[i].x : (mid ? xa[i].x : T(0));
    Cc[pl][2 * par][t][2 * c2 + 1] = pair ? xa[i].y + xb[i].y : (mid ? xa[i].y : T(0));
    Cc[pl][2 * par + 1][t][2 * c2] = pair ? xa[i].x - xb[i].x : T(0);
    Cc[pl][2 * par + 1][t][2 * c2 + 1] = pair ? xa[i].y - xb[i].y : T(0);
  }
  {
    const double* ax_tab = f.axis == 1 ? tmu2 : tmu3;
    for (int i = tid; i < P; i += NT) tax[i] = ax_tab[i];
  }
  // column position and the divisor terms that do not depend on the row
  // (loaded here, ahead of the forward product)
  const int dl = d0 + lr;
  int i1, i2, i3;
  if (f.axis == 1) { i1 = dl; i2 = 0; i3 = o; }
  else { i1 = dl % f.P1; i2 = dl / f.P1; i3 = 0; }
  const bool dvalid = i1 < f.m1 && i2 < f.m2 && i3 < f.m3;
  const double cst = f.axis == 1 ? tmu1[dl] + (tmu3 ? tmu3[o] : 0.0)
                                 : tmu1[dl % f.P1] + tmu2[dl / f.P1];
  const double lre = lam[2 * k], lim = lam[2 * k + 1];
  const double lre1 = real_pair ? lam[2 * f.nk] : 0.0;
  __syncthreads();

  V acc[4][2];
  auto clear = [&]() {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = V{0, 0, 0, 0};
  };
  // one quarter-product pass over all t from the staged operands; table
  // fragments come from L2 through a three-slot register ring, loaded two K
  // steps ahead of the matrix-core work (the loop is unrolled so the ring
  // slots are fixed registers and no copy waits for a load in flight)
  auto load_a = [&](int ks, T (&a)[4]) {
    const int t = 4 * ks + lk;
#pragma unroll
    for (int tb = 0; tb < 4; ++tb) a[tb] = tt[((int64_t)tb * HQ + t) * HQ + q0 + lr];
  };
  auto product = [&]() {
    constexpr int NK = HQ / 4;
    clear();
    T ring[3][4];
    load_a(0, ring[0]);
    load_a(1, ring[1]);
#pragma unroll
    for (int ks = 0; ks < NK; ++ks) {
      const int t = 4 * ks + lk;
      if (ks + 2 < NK) load_a(ks + 2, ring[(ks + 2) % 3]);
      T b[2][2][2];   // b[pl][par][sign]
#pragma unroll
      for (int pl = 0; pl < 2; ++pl)
#pragma unroll
        for (int par = 0; par < 2; ++par) {
          b[pl][par][0] = Cc[pl][2 * par][t][lr];
          b[pl][par][1] = Cc[pl][2 * par + 1][t][lr];
        }
#pragma unroll
      for (int tb = 0; tb < 4; ++tb)
#pragma unroll
        for (int pl = 0; pl < 2; ++pl)
          acc[tb][pl] = Mf<T>::mfma(ring[ks % 3][tb], b[pl][tb >> 1][tb & 1], acc[tb][pl]);
    }
  };

  // ---- forward product
  product();

  // in T arithmetic, the FP64 divisor terms rounded to T (as the unfused
  // FP32 epilogue does)
  auto divide = [&](T& vr, T& vi, int a) {
    if (!dvalid) { vr = T(0); vi = T(0); return; }
    const double mu = cst + tax[a];
    if (real_pair) {
      vr = vr / (T)(lre + mu);
      vi = vi / (T)(lre1 + mu);
    } else {
      const T cc = (T)(lre + mu), dd = (T)lim;
      const T inv = T(1) / (cc * cc + dd * dd);
      const T nr = (vr * cc + vi * dd) * inv;
      const T ni = (vi * cc - vr * dd) * inv;
      vr = nr;
      vi = ni;
    }
    if (f.ims_r) {   // Q1 elements: B_k = M (lambda_k I + tau M^{-1} K), sine basis
      const T ms = (T)(f.ims_c[dl] * f.ims_r[a]);
      vr *= ms;
      vi *= ms;
    }
  };
  // epilogue -> divide -> inverse inputs, held in registers until the tile is free
  T cmb[4][2][4];   // [v][plane][combo u+, u-, v+, v-]
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int q = q0 + Mf<T>::row(lk, v);
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      const int r = 2 * q + s2;   // s2 = 0: even pair (u), 1: odd pair (v)
      const int rb = m - 1 - r;
      T tr = T(0), ti = T(0), br = T(0), bi = T(0);   // top row r and bottom row rb
      if (r < h) {
        const T ore = acc[s2][0][v], ere = acc[2 + s2][0][v];
        const T oim = acc[s2][1][v], eim = acc[2 + s2][1][v];
        tr = ore + ere;
        ti = oim + eim;
        divide(tr, ti, r);
        if (rb > r) {
          br = ore - ere;
          bi = oim - eim;
          divide(br, bi, rb);
        }
      }
      // pair (r, rb): + and -; the middle (rb == r) keeps y_r alone in +
      const bool pair = r < h && rb > r, mid = r < h && rb == r;
      cmb[v][0][2 * s2] = pair ? tr + br : (mid ? tr : T(0));
      cmb[v][0][2 * s2 + 1] = pair ? tr - br : T(0);
      cmb[v][1][2 * s2] = pair ? ti + bi : (mid ? ti : T(0));
      cmb[v][1][2 * s2 + 1] = pair ? ti - bi : T(0);
    }
  }
  __syncthreads();   // every wave is done reading the forward operands
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int pl = 0; pl < 2; ++pl)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) Cc[pl][cb][q0 + Mf<T>::row(lk, v)][lr] = cmb[v][pl][cb];
  __syncthreads();

  // ---- inverse product and output rows
  product();
  T* ob0 = out + base0;
  T* ob1 = out + base1;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int q = q0 + Mf<T>::row(lk, v);
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      const int r = 2 * q + s2, rb = m - 1 - r;
      if (r >= h) continue;
      const T ore = acc[s2][0][v], ere = acc[2 + s2][0][v];
      const T oim = acc[s2][1][v], eim = acc[2 + s2][1][v];
      const int64_t offt = (int64_t)r * f.R + dl, offb = (int64_t)rb * f.R + dl;
      ob0[offt] = dvalid ? ore + ere : T(0);
      ob1[offt] = dvalid ? oim + eim : T(0);
      if (rb > r) {
        ob0[offb] = dvalid ? ore - ere : T(0);
        ob1[offb] = dvalid ? oim - eim : T(0);
      }
    }
  }
  // padding rows m .. P-1 of this column tile
  for (int e = tid; e < 2 * (P - m) * FCF; e += NT) {
    const int pl = e / ((P - m) * FCF), rem = e % ((P - m) * FCF);
    (pl ? ob1 : ob0)[(int64_t)(m + rem / FCF) * f.R + d0 + rem % FCF] = T(0);
  }
}

// ---------------------------------------------------------------- rows kernel (x axis)
// Along x, the contiguous axis, for FP64 with odd m and P = 4 HQ: a block owns
// 16 whole x-rows of one plane pair.  Loads run along the rows; element j of
// a row (j = 2t + par < P/2) pairs with its mirror m-1-j, the fold's + and -
// operands are formed in registers and stored in LDS as [combo][row][t]; the
// matrix cores take the data as the A operand (16 rows x 4 t) and the
// transposed quarter tables as B, so the outputs come out row-major and go
// back through LDS for stores that also run along the rows.  S is its own
// inverse, so the kernel serves the forward and the inverse product.
// LDS strides: operand rows HQ + 2 apart and operand planes 8 elements more
// than a multiple of 32, so that the staging stores and the MFMA operand reads
// of a half-wave fall on distinct banks; output rows P + 1 apart likewise.
template <int HQ>
__global__ __launch_bounds__(64 * (HQ / 16)) __attribute__((amdgpu_waves_per_eu(2))) void k_dst_fold2_rows(
    const double* in, double* out, const double* __restrict__ tt,
    FoldArgs f, int ntiles) {
  using V = d4;
  constexpr int P = 4 * HQ, NT = 64 * (HQ / 16), NV = 16;
  constexpr int S = HQ + 2, PLS = NV * S + 8, YS = P + 1;
  constexpr int OPS = 2 * 4 * PLS, OUTS = 2 * NV * YS;
  static_assert(NT == P, "one thread per row element in the store loop, two rows per load step");
  __shared__ double lds[OPS > OUTS ? OPS : OUTS];
  auto cc = [&](int pl, int cb, int v, int t) -> double& { return lds[(pl * 4 + cb) * PLS + v * S + t]; };
  auto yy = [&](int pl, int v, int a) -> double& { return lds[(pl * NV + v) * YS + a]; };

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int m = f.m, h = (m + 1) / 2, q0 = w * 16;

  // tile b: rows d0 .. d0 + 15 (d0 = 16 (b % ndt)) of frequency block k = b / ndt
  auto bases = [&](int b, int& d0, int64_t& base0, int64_t& base1) {
    const int k = b / f.ndt;
    d0 = (b % f.ndt) * NV;
    base0 = (int64_t)k * 2 * f.PS;
    base1 = (f.packed && k == 0) ? (int64_t)f.nk * 2 * f.PS : base0 + f.PS;
  };
  // element j < P/2 of a row (j = 2t + par) pairs with its mirror m-1-j; the
  // next tile's raw values are loaded while the current tile is processed
  // Thread tid takes element j = tid % (P/2) of rows v = tid / (P/2) + 2 i'
  // (NT = P: two rows per step), plane pl = i / (NST/2): a per-lane offset plus
  // wave-uniform ones, so no per-row 64-bit offsets stay live across tiles.
  constexpr int NST = 2 * NV * (P / 2) / NT;   // (pl, row pair) steps per thread
  const int jl = tid % (P / 2), vl = tid / (P / 2);
  const int jml = m - 1 - jl, jcl = jml > jl ? jml : jl;   // mirror, in range either way
  double xa[NST], xb[NST];
  auto load = [&](int b) {
    int d0;
    int64_t base0, base1;
    bases(b, d0, base0, base1);
    const double* row = in + (int64_t)(d0 + vl) * f.R;
#pragma unroll
    for (int i = 0; i < NST; ++i) {
      const double* src = row + (i < NST / 2 ? base0 : base1) + (int64_t)(2 * (i % (NST / 2))) * f.R;
      xa[i] = src[jl];
      xb[i] = src[jcl];
    }
  };
  auto load_b = [&](int ks, double (&bq)[4]) {
    const int t = 4 * ks + lk;
#pragma unroll
    for (int tb = 0; tb < 4; ++tb) bq[tb] = tt[((int64_t)tb * HQ + t) * HQ + q0 + lr];
  };

  const StripRange sr = xcd_strips(ntiles);
  if (sr.first < sr.end) load(sr.first);
  for (int b = sr.first; b < sr.end; b += sr.step) {
    int d0;
    int64_t base0, base1;
    bases(b, d0, base0, base1);
    __syncthreads();   // the previous tile's stores have read the LDS
    {
      // a proper pair gives + and -; the middle (jm = j) keeps x alone in +;
      // beyond the pairs both are zero (those elements are other j's mirrors)
      const int t = jl >> 1, par = jl & 1;
      const bool pair = jml > jl, mid = jml == jl;
#pragma unroll
      for (int i = 0; i < NST; ++i) {
        const int v = vl + 2 * (i % (NST / 2)), pl = i / (NST / 2);
        cc(pl, 2 * par, v, t) = pair ? xa[i] + xb[i] : (mid ? xa[i] : 0.0);
        cc(pl, 2 * par + 1, v, t) = pair ? xa[i] - xb[i] : 0.0;
      }
    }
    if (b + sr.step < sr.end) load(b + sr.step);
    __syncthreads();

    // quarter products: acc[tb][pl] = data(combo tb) x table tb; table
    // fragments through a two-slot register ring one K step ahead (the loop
    // is unrolled by two so the slots are fixed registers)
    V acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c) acc[a][c] = V{0, 0, 0, 0};
    {
      constexpr int NK = HQ / 4;
      static_assert(NK % 2 == 0, "ring of two");
      double ring[2][4];
      load_b(0, ring[0]);
#pragma unroll 2
      for (int ks = 0; ks < NK; ++ks) {
        const int t = 4 * ks + lk;
        if (ks + 1 < NK) load_b(ks + 1, ring[(ks + 1) % 2]);
        double a[2][4];   // a[pl][combo]
#pragma unroll
        for (int pl = 0; pl < 2; ++pl)
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) a[pl][cb] = cc(pl, cb, lr, t);
#pragma unroll
        for (int tb = 0; tb < 4; ++tb)
#pragma unroll
          for (int pl = 0; pl < 2; ++pl)
            acc[tb][pl] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[pl][tb], ring[ks % 2][tb],
                                                               acc[tb][pl], 0, 0, 0);
      }
    }
    __syncthreads();   // every wave is done reading the operands

    // epilogue: lane element i is row v = lk + 4 i, quarter index q = q0 + lr;
    // output r = 2q + s2 takes tables s2 (O) and 2 + s2 (E): y_r = O + E,
    // y_{m-1-r} = O - E
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int v = lk + 4 * i, q = q0 + lr;
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        const int r = 2 * q + s2, rb = m - 1 - r;
        if (r >= h) continue;
#pragma unroll
        for (int pl = 0; pl < 2; ++pl) {
          const double O = acc[s2][pl][i], E = acc[2 + s2][pl][i];
          yy(pl, v, r) = O + E;
          if (rb > r) yy(pl, v, rb) = O - E;
        }
      }
    }
    __syncthreads();

    // stores along the rows (thread tid writes element a = tid of every row);
    // padding positions and rows outside the grid get zero.  The 16 rows of a
    // tile share i3 (P2 is a multiple of 16).
    double* ob0 = out + base0;
    double* ob1 = out + base1;
    const int i2_0 = d0 % f.P2, i3 = d0 / f.P2;
    const bool avalid = tid < m && i3 < f.m3;
#pragma unroll
    for (int it = 0; it < 2 * NV; ++it) {
      const int v = it % NV, pl = it / NV;
      const bool valid = avalid && i2_0 + v < f.m2;
      (pl ? ob1 : ob0)[(int64_t)(d0 + v) * f.R + tid] = valid ? yy(pl, v, tid) : 0.0;
    }
  }
}

}  // namespace

template <typename T>
hipError_t launch_dst_fold(const T* in, T* out, const T* Soe, const T* Soo, const FoldArgs& f,
                           bool left, const double* lam, const double* tmu1, const double* tmu2,
                           const double* tmu3, hipStream_t s) {
  if (f.Hp % 32 || f.Hp < 32 || f.ndt < 1 || f.nout < 1 || f.nk < 1) return hipErrorInvalidValue;
  if (f.m < 1 || f.m > 2 * f.Hp) return hipErrorInvalidValue;
  if (f.Hp % 64 == 0)
    return launch_fold_fr<T, 64>(in, out, Soe, Soo, f, left, lam, tmu1, tmu2, tmu3, s);
  return launch_fold_fr<T, 32>(in, out, Soe, Soo, f, left, lam, tmu1, tmu2, tmu3, s);
}

template <typename T>
hipError_t launch_dst_fold2(const T* in, T* out, const T* tabs, const FoldArgs& f, bool left,
                            const double* lam, const double* tmu1, const double* tmu2,
                            const double* tmu3, hipStream_t s) {
  if (f.m % 2 == 0 || f.Hp % 64 || f.Hp < 64 || (f.m + 1) / 2 > f.Hp || f.ndt < 1 ||
      f.nout < 1 || f.nk < 1)
    return hipErrorInvalidValue;
  return launch_fold2<T>(in, out, tabs, f, left, lam, tmu1, tmu2, tmu3, s);
}

template <typename T>
hipError_t launch_dst_fold2_fused(const T* in, T* out, const T* tt, const FoldArgs& f,
                                  const double* lam, const double* tmu1, const double* tmu2,
                                  const double* tmu3, hipStream_t s) {
  const int P = 2 * f.Hp;
  if (f.m % 2 == 0 || (P != 128 && P != 256) || (f.m + 1) / 2 > f.Hp || f.ndt < 1 ||
      f.nout < 1 || f.nk < 1 || (f.axis != 1 && f.axis != 2) || !lam)
    return hipErrorInvalidValue;
  const int64_t nblk = (int64_t)f.ndt * f.nout * f.nk;
  if (nblk > 0x7fffffff) return hipErrorInvalidConfiguration;
  if (P == 256)
    hipLaunchKernelGGL((k_dst_fold2_fused<T, 64>), dim3((unsigned)nblk), dim3(256), 0, s, in, out,
                       tt, f, lam, tmu1, tmu2, tmu3);
  else
    hipLaunchKernelGGL((k_dst_fold2_fused<T, 32>), dim3((unsigned)nblk), dim3(128), 0, s, in, out,
                       tt, f, lam, tmu1, tmu2, tmu3);
  return hipGetLastError();
}
template hipError_t launch_dst_fold2_fused<double>(const double*, double*, const double*,
                                                   const FoldArgs&, const double*, const double*,
                                                   const double*, const double*, hipStream_t);
template hipError_t launch_dst_fold2_fused<float>(const float*, float*, const float*,
                                                  const FoldArgs&, const double*, const double*,
                                                  const double*, const double*, hipStream_t);

hipError_t launch_dst_fold2_rows(const double* in, double* out, const double* tt,
                                 const FoldArgs& f, hipStream_t s) {
  const int P = 2 * f.Hp;
  if (f.m % 2 == 0 || (P != 128 && P != 256) || f.m > P || f.R != P || f.axis != 0 ||
      f.ndt < 1 || f.nk < 1 || f.P2 < 1 || f.P2 % 16)
    return hipErrorInvalidValue;
  const int64_t ntiles = (int64_t)f.ndt * f.nk;
  if (ntiles > 0x7fffffff) return hipErrorInvalidConfiguration;
  if (P == 256) {
    static const int resident = persistent_grid(k_dst_fold2_rows<64>, 256);
    if (resident < 8) return hipErrorInvalidDeviceFunction;
    hipLaunchKernelGGL((k_dst_fold2_rows<64>), dim3(strip_grid(resident, ntiles)), dim3(256), 0,
                       s, in, out, tt, f, (int)ntiles);
  } else {
    static const int resident = persistent_grid(k_dst_fold2_rows<32>, 128);
    if (resident < 8) return hipErrorInvalidDeviceFunction;
    hipLaunchKernelGGL((k_dst_fold2_rows<32>), dim3(strip_grid(resident, ntiles)), dim3(128), 0,
                       s, in, out, tt, f, (int)ntiles);
  }
  return hipGetLastError();
}

hipError_t launch_dst_fold_bf16x3(const float* in, float* out, const uint16_t* const* tabs,
                                  const FoldArgs& f, bool left, const double* lam,
                                  const double* tmu1, const double* tmu2, const double* tmu3,
                                  hipStream_t s) {
  if (f.Hp % 32 || f.Hp < 32 || f.ndt < 1 || f.nout < 1 || f.nk < 1 || 2 * f.Hp > 1024)
    return hipErrorInvalidValue;
  if (f.m < 1 || f.m > 2 * f.Hp) return hipErrorInvalidValue;
  for (int i = 0; i < 4; ++i)
    if (!tabs[i]) return hipErrorInvalidValue;
  if (f.Hp % 64 == 0)
    return launch_fold_bf3_fr<64>(in, out, tabs, f, left, lam, tmu1, tmu2, tmu3, s);
  return launch_fold_bf3_fr<32>(in, out, tabs, f, left, lam, tmu1, tmu2, tmu3, s);
}

template hipError_t launch_dst_fold2<double>(const double*, double*, const double*,
                                             const FoldArgs&, bool, const double*,
                                             const double*, const double*, const double*,
                                             hipStream_t);
template hipError_t launch_dst_fold2<float>(const float*, float*, const float*,
                                            const FoldArgs&, bool, const double*,
                                            const double*, const double*, const double*,
                                            hipStream_t);

template hipError_t launch_dst_fold<double>(const double*, double*, const double*, const double*,
                                            const FoldArgs&, bool, const double*, const double*,
                                            const double*, const double*, hipStream_t);
template hipError_t launch_dst_fold<float>(const float*, float*, const float*, const float*,
                                           const FoldArgs&, bool, const double*, const double*,
                                           const double*, const double*, hipStream_t);

}  // namespace aao
