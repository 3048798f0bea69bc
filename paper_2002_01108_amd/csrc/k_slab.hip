// Both in-plane DST-I products of a 3D spectrum in one pass (constant
// coefficient Step 2, Section 4, eq. (blockdiaginv)).
// This file is compiled with the MFMA results in VGPRs (build.py): left to
// its default the compiler keeps them in AGPRs here and copies the loop
// accumulators between the two register files on every K step.
#include "common.h"

namespace aao {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Both in-plane products of a 3D spectrum (x and y, P1 = P2 = 128, odd m1 and
// m2 with the same quarter tables) in one pass: a z slab of one plane
// (128 x 128 FP64 = 128 KB) sits in LDS while the x product (rows) and then
// the y product (columns) run on it, so the spectrum crosses HBM once for two
// products instead of twice.  The two products commute (S_y X S_x), so the
// same launch serves the forward and the inverse sweep.  Both use the second
// fold: element j = 2t + par < 64 of a row (column) pairs with its mirror
// m-1-j into x_j +- x_{m-1-j} (the middle keeps x_j alone in +, beyond the
// pairs both are zero), the quarter tables ([4][32][32]: A+, A-, B+, B-)
// multiply them, and output r = 2q + s2 < h takes O = table s2 and
// E = table 2 + s2: y_r = O + E, y_{m-1-r} = O - E.
// LDS: the slab (128 KB; element (row, col) at row * 128 + (col ^ (row & 15)),
// so that 16 rows of one column, as well as 16 columns of one row, fall on
// distinct banks) and the tables (32 KB, loaded once per block, swizzled the
// same way): 160 KB, one block per CU.  No global load in the K loops: a table wait there would also
// wait for the next slab's prefetch (the vector memory counter is in order).
// A block of 8 waves (two per SIMD, so that one wave's matrix-core work covers
// the other's LDS latency) walks slabs (xcd_strips): it stages the slab
// prefetched into registers, loads the next one while it computes, and
// writes the result back in place.  Phase x: wave w owns rows 16w .. 16w+15
// (the data as the MFMA A operand, the table as B); phase y: wave w owns
// columns 16w .. 16w+15 (the table as A, the data as B).  A wave reads and
// writes only its own rows (columns) within a phase, so one barrier separates
// the phases.  Padding (rows >= m2, columns >= m1) must be zero on input and
// stays zero.
// FP32 (the FP32 preconditioner): the same with v_mfma_f32_16x16x4f32, 80 KB of
// LDS (74 KB on the third fold; two blocks per CU), the slab swizzled by (row & 15) << 3 (64 banks of
// 32-bit words: the 16 rows of a fragment read land in pairs on 32 banks) and
// the tables transposed ([tb][t][q], q contiguous, q ^ 16 ((t >> 1) & 1)).
// Third fold (m1 = m2 = 127, so m + 1 = 128 is a multiple of 4): with
// the quarter products written over output index q and pair index t (outputs
// r = 2q + s, elements j = 2t + b), three of the four split again.  For r odd
// (r + 1 = 2a) the element pairs j <-> j' = 62 - j (of either parity b; the
// odd elements j = 2t + 1 pair with 61 - 2t), i.e. J = j + 1 <-> 64 - J, have
// S_{r,j'} = (-1)^{a+1} S_{r,j}: the minus
// combinations q_j = x_j - x_{126-j} fold once more into q_j +- q_{j'}, the
// sign set by q's parity (16 x 16 products instead of 32 x 32).  For r even
// and j odd the outputs pair: S_{62-r, j} = (-1)^t S_{r,j} (j = 2t + 1), so
// the plus product splits into its even-t and odd-t halves Ev, Od with
// E_r = Ev + Od and E_{62-r} = Ev - Od.  The remaining r even, j even product
// (a DST-IV of size 32) keeps its 32 x 32 form.  Tables ([q][kappa], built on
// the host): T0 32 x 32 (A+: rows q < 16 give r = 2q, rows 16 + i give
// r = 62 - 2i; kappa < 16 takes j = 2 kappa, kappa >= 16 j = 94 - 2 kappa),
// then six 16 x 16: A- for r = 4q + 1 and 4q + 3 over j = 2 kappa, B- for the
// same rows over j = 2 kappa + 1 (kappa = 15 is j = 31 paired with itself:
// halved, its combination comes out doubled), B+ Ev and Od for r = 2q over
// j = 4 kappa + 1 and 4 kappa + 3 (kappa = 15 is the middle element j = 63:
// halved likewise).  Lane q (phase x: lane row lr; phase y: output row) then
// owns r = 2q, 62 - 2q, 4q + 1, 4q + 3 and their mirrors 126 - r.  40 MFMAs per
// 16 lines and product instead of 64.
constexpr int XYP = 128, XYQ = 32;
constexpr int F3N = 32 * 32 + 6 * 16 * 16;   // third-fold table entries

template <typename T> struct Slab;
template <> struct Slab<double> {
  typedef d4 V;
  typedef double2 T2;
  static __device__ __forceinline__ V mfma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of accumulator element v (16x16 FP64 output layout)
  static __device__ __forceinline__ int orow(int lk, int v) { return lk + 4 * v; }
  static __device__ __forceinline__ int at(int row, int col) {
    return row * XYP + (col ^ (row & 15));
  }
  // tables stored [tb][q][t ^ (q & 15)] from the [tb][q][t] FP64 quarter tables
  static __device__ __forceinline__ int tab_at(int tb, int q, int t) {
    return (tb * XYQ + q) * XYQ + (t ^ (q & 15));
  }
  static __device__ __forceinline__ int tab_src(int tb, int q, int t) {
    return (tb * XYQ + q) * XYQ + t;
  }
  // third-fold tables: T0 row q (< 32), column k; table tb of the six
  // 16 x 16 ones, row q, column k (16 rows of one column on distinct banks)
  static __device__ __forceinline__ int t0_at(int q, int k) { return q * XYQ + (k ^ (q & 15)); }
  static __device__ __forceinline__ int t16_at(int tb, int q, int k) {
    return XYQ * XYQ + tb * 256 + q * 16 + (k ^ q);
  }
};
template <> struct Slab<float> {
  typedef f4 V;
  typedef float2 T2;
  static __device__ __forceinline__ V mfma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int orow(int lk, int v) { return 4 * lk + v; }
  static __device__ __forceinline__ int at(int row, int col) {
    return row * XYP + (col ^ ((row & 15) << 3));
  }
  // tables stored [tb][t][q ^ 16 ((t >> 1) & 1)] from the [tb][t][q] FP32 ones
  static __device__ __forceinline__ int tab_at(int tb, int q, int t) {
    return (tb * XYQ + t) * XYQ + (q ^ (((t >> 1) & 1) << 4));
  }
  static __device__ __forceinline__ int tab_src(int tb, int q, int t) {
    return (tb * XYQ + t) * XYQ + q;
  }
  // third-fold tables, columns XOR-swizzled by multiples of 4 so that a
  // fragment read (16 rows q x 4 consecutive columns) hits 64 distinct banks
  static __device__ __forceinline__ int t0_at(int q, int k) {
    return q * XYQ + (k ^ (4 * ((q >> 1) & 7)));
  }
  static __device__ __forceinline__ int t16_at(int tb, int q, int k) {
    return XYQ * XYQ + tb * 256 + q * 16 + (k ^ (4 * (q >> 2)));
  }
};

template <typename F, bool L3>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(F) == 8 ? 2 : 4)))
void k_dst_xy(F* __restrict__ spec, const F* __restrict__ tab, SlabArgs a) {
  using S = Slab<F>;
  using V = typename S::V;
  using T2 = typename S::T2;
  __shared__ F X[XYP * XYP];
  __shared__ F T[L3 ? F3N : 4 * XYQ * XYQ];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // lane coordinates of the MFMA fragments, renewed opaquely for every slab
  // (below) so that the compiler does not hoist the phases' per-lane
  // addresses and store masks out of the slab loop and hold them in registers
  int lr = lane & 15, lk = lane >> 4;
  const int nslab = a.nk * 2 * a.m3;
  const int64_t zs = (int64_t)XYP * XYP;   // one z slab of a plane

  // tables, swizzled so that the 16 q rows of a fragment read fall on distinct banks
  if constexpr (L3) {
    for (int i = tid; i < F3N; i += 512) {
      if (i < XYQ * XYQ) {
        T[S::t0_at(i / XYQ, i % XYQ)] = tab[i];
      } else {
        const int e = i - XYQ * XYQ;
        T[S::t16_at(e / 256, (e / 16) % 16, e % 16)] = tab[i];
      }
    }
  } else {
    for (int i = tid; i < 4 * XYQ * XYQ; i += 512) {
      const int tb = i / (XYQ * XYQ), q = (i / XYQ) % XYQ, t = i % XYQ;
      T[S::tab_at(tb, q, t)] = tab[S::tab_src(tb, q, t)];
    }
  }
  // third-fold fragments: T0 row q (< 32), column kappa; table tb of the six
  // 16 x 16 ones, row q (< 16), column kappa
  auto t0 = [&](int q, int k) { return T[S::t0_at(q, k)]; };
  auto t16 = [&](int tb, int q, int k) { return T[S::t16_at(tb, q, k)]; };

  auto slab_base = [&](int s) -> int64_t {
    const int z = s % a.m3, rest = s / a.m3, pl = rest & 1, k = rest >> 1;
    const int64_t b0 = (int64_t)k * 2 * a.PS;
    const int64_t b = pl ? ((a.packed && k == 0) ? (int64_t)a.nk * 2 * a.PS : b0 + a.PS) : b0;
    return b + (int64_t)z * zs;
  };
  // thread -> rows w + 8 i (i < 16), columns 2 lane, 2 lane + 1: a wave-uniform
  // row address plus one per-lane offset, so no per-row address registers
  const int loff = w * (XYP / 2) + lane;   // in two-element vectors
  T2 pf[16];
  auto load = [&](int s) {
    const F* sb = spec + slab_base(s);
#pragma unroll
    for (int i = 0; i < 16; ++i) pf[i] = reinterpret_cast<const T2*>(sb + (int64_t)8 * i * XYP)[loff];
  };
  // table fragment: lane (lr, lk) takes table tb at q = 16 qt + lr, t = 4 ks + lk
  auto tfrag = [&](int tb, int qt, int ks) { return T[S::tab_at(tb, 16 * qt + lr, 4 * ks + lk)]; };
  // combos of element j with its mirror m-1-j (x_j, x_m: their values)
  auto combo = [](int j, int m, F xj, F xm, F& p, F& q) {
    const int jm = m - 1 - j;
    p = jm > j ? xj + xm : (jm == j ? xj : F(0));
    q = jm > j ? xj - xm : F(0);
  };

  const StripRange sr = xcd_strips(nslab);
  if (sr.first < sr.end) load(sr.first);
  for (int s = sr.first; s < sr.end; s += sr.step) {
    int lo = lane;
    asm volatile("" : "+v"(lo));
    lr = lo & 15;
    lk = lo >> 4;
    __syncthreads();   // the previous slab's stores have read X (and T is in place)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = w + 8 * i;
      X[S::at(row, 2 * lane)] = pf[i].x;
      X[S::at(row, 2 * lane + 1)] = pf[i].y;
    }
    if (s + sr.step < sr.end) load(s + sr.step);
    __syncthreads();

    // ---- phase x: rows R0 .. R0 + 15 (rows are independent: a tile's
    // outputs replace its inputs once its K loop is done)
    if constexpr (L3) {
      const int R0 = 16 * w, row = R0 + lr;
      auto xr = [&](int j) { return X[S::at(row, j)]; };
      V aP0{0, 0, 0, 0}, aP1{0, 0, 0, 0}, aMe{0, 0, 0, 0}, aMo{0, 0, 0, 0};
      V bMe{0, 0, 0, 0}, bMo{0, 0, 0, 0}, bEv{0, 0, 0, 0}, bOd{0, 0, 0, 0};
#pragma unroll 2
      for (int ks = 0; ks < 4; ++ks) {
        const int t = 4 * ks + lk;
        const F xa = xr(2 * t), xb = xr(126 - 2 * t), xc = xr(62 - 2 * t), xd = xr(64 + 2 * t);
        const F xe = xr(2 * t + 1), xf = xr(125 - 2 * t), xg = xr(61 - 2 * t), xh = xr(65 + 2 * t);
        const F xi = xr(4 * t + 1), xj = xr(125 - 4 * t), xk = xr(4 * t + 3), xl = xr(123 - 4 * t);
        const F pA0 = xa + xb, qA0 = xa - xb, pA1 = xc + xd, qA1 = xc - xd;
        const F qB0 = xe - xf, qB1 = xg - xh;
        aP0 = S::mfma(pA0, t0(lr, t), aP0);
        aP1 = S::mfma(pA0, t0(16 + lr, t), aP1);
        aP0 = S::mfma(pA1, t0(lr, 16 + t), aP0);
        aP1 = S::mfma(pA1, t0(16 + lr, 16 + t), aP1);
        aMe = S::mfma(qA0 + qA1, t16(0, lr, t), aMe);
        aMo = S::mfma(qA0 - qA1, t16(1, lr, t), aMo);
        bMe = S::mfma(qB0 + qB1, t16(2, lr, t), bMe);
        bMo = S::mfma(qB0 - qB1, t16(3, lr, t), bMo);
        bEv = S::mfma(xi + xj, t16(4, lr, t), bEv);
        bOd = S::mfma(xk + xl, t16(5, lr, t), bOd);
      }
      // lane element v: row R0 + orow(lk, v), output rows of q = lr
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int orow = R0 + S::orow(lk, v);
        const F E0 = bEv[v] + bOd[v], E1 = bEv[v] - bOd[v];
        X[S::at(orow, 2 * lr)] = aP0[v] + E0;
        X[S::at(orow, 126 - 2 * lr)] = aP0[v] - E0;
        X[S::at(orow, 62 - 2 * lr)] = aP1[v] + E1;
        X[S::at(orow, 64 + 2 * lr)] = aP1[v] - E1;
        X[S::at(orow, 4 * lr + 1)] = aMe[v] + bMe[v];
        X[S::at(orow, 125 - 4 * lr)] = aMe[v] - bMe[v];
        X[S::at(orow, 4 * lr + 3)] = aMo[v] + bMo[v];
        if (lr < 15) X[S::at(orow, 123 - 4 * lr)] = aMo[v] - bMo[v];
      }
    } else {
      const int m = a.m1, h = (m + 1) / 2, R0 = 16 * w;
      V acc[4][2];   // [table][q tile]
#pragma unroll
      for (int tb = 0; tb < 4; ++tb)
#pragma unroll
        for (int qt = 0; qt < 2; ++qt) acc[tb][qt] = V{0, 0, 0, 0};
      const int row = R0 + lr;
#pragma unroll 2
      for (int ks = 0; ks < 8; ++ks) {
        const int t = 4 * ks + lk;
        F op[4];
#pragma unroll
        for (int par = 0; par < 2; ++par) {
          const int j = 2 * t + par;
          combo(j, m, X[S::at(row, j)], X[S::at(row, m - 1 - j)], op[2 * par], op[2 * par + 1]);
        }
#pragma unroll
        for (int tb = 0; tb < 4; ++tb)
#pragma unroll
          for (int qt = 0; qt < 2; ++qt) acc[tb][qt] = S::mfma(op[tb], tfrag(tb, qt, ks), acc[tb][qt]);
      }
      // lane element v: row R0 + orow(lk, v), quarter index q = 16 qt + lr:
      // outputs r = 2 q + s2 and m-1-r of that row
#pragma unroll
      for (int qt = 0; qt < 2; ++qt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int s2 = 0; s2 < 2; ++s2) {
            const int orow = R0 + S::orow(lk, v);
            const int r = 2 * lr + 32 * qt + s2, rb = m - 1 - r;
            const F O = acc[s2][qt][v], E = acc[2 + s2][qt][v];
            if (r < h) X[S::at(orow, r)] = O + E;
            if (r < h && rb > r) X[S::at(orow, rb)] = O - E;
          }
    }
    __syncthreads();
    // ---- phase y: columns C0 .. C0 + 15 (columns are independent)
    if constexpr (L3) {
      const int C0 = 16 * w, col = C0 + lr;
      auto xr = [&](int j) { return X[S::at(j, col)]; };
      V aP0{0, 0, 0, 0}, aP1{0, 0, 0, 0}, aMe{0, 0, 0, 0}, aMo{0, 0, 0, 0};
      V bMe{0, 0, 0, 0}, bMo{0, 0, 0, 0}, bEv{0, 0, 0, 0}, bOd{0, 0, 0, 0};
#pragma unroll 2
      for (int ks = 0; ks < 4; ++ks) {
        const int t = 4 * ks + lk;
        const F xa = xr(2 * t), xb = xr(126 - 2 * t), xc = xr(62 - 2 * t), xd = xr(64 + 2 * t);
        const F xe = xr(2 * t + 1), xf = xr(125 - 2 * t), xg = xr(61 - 2 * t), xh = xr(65 + 2 * t);
        const F xi = xr(4 * t + 1), xj = xr(125 - 4 * t), xk = xr(4 * t + 3), xl = xr(123 - 4 * t);
        const F pA0 = xa + xb, qA0 = xa - xb, pA1 = xc + xd, qA1 = xc - xd;
        const F qB0 = xe - xf, qB1 = xg - xh;
        aP0 = S::mfma(t0(lr, t), pA0, aP0);
        aP1 = S::mfma(t0(16 + lr, t), pA0, aP1);
        aP0 = S::mfma(t0(lr, 16 + t), pA1, aP0);
        aP1 = S::mfma(t0(16 + lr, 16 + t), pA1, aP1);
        aMe = S::mfma(t16(0, lr, t), qA0 + qA1, aMe);
        aMo = S::mfma(t16(1, lr, t), qA0 - qA1, aMo);
        bMe = S::mfma(t16(2, lr, t), qB0 + qB1, bMe);
        bMo = S::mfma(t16(3, lr, t), qB0 - qB1, bMo);
        bEv = S::mfma(t16(4, lr, t), xi + xj, bEv);
        bOd = S::mfma(t16(5, lr, t), xk + xl, bOd);
      }
      // lane element v: output rows of q = orow(lk, v), column C0 + lr
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int q = S::orow(lk, v);
        const F E0 = bEv[v] + bOd[v], E1 = bEv[v] - bOd[v];
        X[S::at(2 * q, col)] = aP0[v] + E0;
        X[S::at(126 - 2 * q, col)] = aP0[v] - E0;
        X[S::at(62 - 2 * q, col)] = aP1[v] + E1;
        X[S::at(64 + 2 * q, col)] = aP1[v] - E1;
        X[S::at(4 * q + 1, col)] = aMe[v] + bMe[v];
        X[S::at(125 - 4 * q, col)] = aMe[v] - bMe[v];
        X[S::at(4 * q + 3, col)] = aMo[v] + bMo[v];
        if (q < 15) X[S::at(123 - 4 * q, col)] = aMo[v] - bMo[v];
      }
    } else {
      const int m = a.m2, h = (m + 1) / 2, C0 = 16 * w;
      V acc[4][2];   // [table][q tile]
#pragma unroll
      for (int tb = 0; tb < 4; ++tb)
#pragma unroll
        for (int qt = 0; qt < 2; ++qt) acc[tb][qt] = V{0, 0, 0, 0};
      const int col = C0 + lr;
#pragma unroll 2
      for (int ks = 0; ks < 8; ++ks) {
        const int t = 4 * ks + lk;
        F op[4];
#pragma unroll
        for (int par = 0; par < 2; ++par) {
          const int j = 2 * t + par;
          combo(j, m, X[S::at(j, col)], X[S::at(m - 1 - j, col)], op[2 * par], op[2 * par + 1]);
        }
#pragma unroll
        for (int tb = 0; tb < 4; ++tb)
#pragma unroll
          for (int qt = 0; qt < 2; ++qt) acc[tb][qt] = S::mfma(tfrag(tb, qt, ks), op[tb], acc[tb][qt]);
      }
      // lane element v: quarter index q = 16 qt + orow(lk, v), column C0 + lr:
      // output rows r = 2 q + s2 and m-1-r of that column
#pragma unroll
      for (int qt = 0; qt < 2; ++qt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int s2 = 0; s2 < 2; ++s2) {
            const int r = 32 * qt + 2 * S::orow(lk, v) + s2, rb = m - 1 - r;
            const F O = acc[s2][qt][v], E = acc[2 + s2][qt][v];
            if (r < h) X[S::at(r, col)] = O + E;
            if (r < h && rb > r) X[S::at(rb, col)] = O - E;
          }
    }
    __syncthreads();
    F* db = spec + slab_base(s);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = w + 8 * i;
      reinterpret_cast<T2*>(db + (int64_t)8 * i * XYP)[loff] =
          T2{X[S::at(row, 2 * lane)], X[S::at(row, 2 * lane + 1)]};
    }
  }
}


// Last-axis forward product, shifted divide and inverse product of a 3D
// spectrum in one in-place pass (P3 = 128, m3 = 127, on the third fold): a
// block owns, for one frequency block k, one y row and one half of the x range
// (64 columns), the (z, x) slices of both planes (2 x 128 x 64 elements: 128 KB
// FP64, 64 KB FP32) in LDS, so the complex divide finds the real and imaginary
// part of every element in the block.  Wave w runs plane w / 4 on columns
// 16 (w % 4) .. + 15 with the phase-y code of the slab kernel (the table as
// the MFMA A operand, the data as B); between the products one pass over the
// slices divides by lambda_k + tau (mu_x + mu_y + mu_z).  Persistent like the
// slab kernel: the next slice pair is prefetched into registers while the
// current one is computed.  Rows (z) >= m3 and columns (x) >= m1 are padding:
// zero on input, zero on output; y rows >= m2 are not visited (zero stays zero).
template <typename F>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
void k_dst_zdiv(F* __restrict__ spec, const F* __restrict__ tab, SlabArgs a,
                const double* __restrict__ lam, const double* __restrict__ tmu1,
                const double* __restrict__ tmu2, const double* __restrict__ tmu3) {
  // FP64 only: in FP32 the four k rows an operand read touches would share
  // 32-bit banks in this unswizzled layout
  static_assert(sizeof(F) == 8, "the z pass is built for FP64");
  using S = Slab<F>;
  using V = typename S::V;
  using T2 = typename S::T2;
  constexpr int XW = 64;                 // columns per slice
  __shared__ F X[2][XYP * XW];           // [plane][z * 64 + x]
  __shared__ F T[F3N];
  __shared__ double tax[XYP];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int pw = w >> 2, cg = w & 3;     // plane and column group of this wave
  int lr = lane & 15, lk = lane >> 4;
  const int nslab = a.nk * a.m2 * 2;

  for (int i = tid; i < F3N; i += 512) {
    if (i < XYQ * XYQ) {
      T[S::t0_at(i / XYQ, i % XYQ)] = tab[i];
    } else {
      const int e = i - XYQ * XYQ;
      T[S::t16_at(e / 256, (e / 16) % 16, e % 16)] = tab[i];
    }
  }
  for (int i = tid; i < XYP; i += 512) tax[i] = tmu3[i];
  auto t0 = [&](int q, int k) { return T[S::t0_at(q, k)]; };
  auto t16 = [&](int tb, int q, int k) { return T[S::t16_at(tb, q, k)]; };

  // slice s: x half xh, y row, frequency block k; plane bases as in the DST
  // products (the packed block pairs the real planes of k = 0 and n/2)
  struct Slice {
    int xh, y, k;
    int64_t b0, b1;
  };
  auto slice = [&](int s) {
    Slice c;
    c.xh = s & 1;
    s >>= 1;
    c.y = s % a.m2;
    c.k = s / a.m2;
    const int64_t off = (int64_t)c.y * XYP + c.xh * XW;
    c.b0 = (int64_t)c.k * 2 * a.PS + off;
    c.b1 = ((a.packed && c.k == 0) ? (int64_t)a.nk * 2 * a.PS : c.b0 - off + a.PS) + off;
    return c;
  };
  // thread -> (plane, z row, column pair): 32 column pairs per row; load i
  // covers rows 16 i + tid / 32 of plane 0 (i < 8) or plane 1 (i >= 8)
  const int cp = tid & 31, rz = tid >> 5;
  const int64_t zs = (int64_t)XYP * XYP;   // z row stride
  T2 pf[16];
  auto load = [&](int s) {
    const Slice c = slice(s);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const F* b = spec + (i < 8 ? c.b0 : c.b1) + (int64_t)(16 * (i & 7) + rz) * zs;
      pf[i] = reinterpret_cast<const T2*>(b)[cp];
    }
  };

  // one product of plane pw on columns 16 cg .. + 15, outputs back into X
  auto product = [&]() {
    const int col = 16 * cg + lr;
    F* xp = X[pw];
    auto xr = [&](int j) { return xp[j * XW + col]; };
    V aP0{0, 0, 0, 0}, aP1{0, 0, 0, 0}, aMe{0, 0, 0, 0}, aMo{0, 0, 0, 0};
    V bMe{0, 0, 0, 0}, bMo{0, 0, 0, 0}, bEv{0, 0, 0, 0}, bOd{0, 0, 0, 0};
#pragma unroll 2
    for (int ks = 0; ks < 4; ++ks) {
      const int t = 4 * ks + lk;
      const F xa = xr(2 * t), xb = xr(126 - 2 * t), xc = xr(62 - 2 * t), xd = xr(64 + 2 * t);
      const F xe = xr(2 * t + 1), xf = xr(125 - 2 * t), xg = xr(61 - 2 * t), xh = xr(65 + 2 * t);
      const F xi = xr(4 * t + 1), xj = xr(125 - 4 * t), xk = xr(4 * t + 3), xl = xr(123 - 4 * t);
      const F pA0 = xa + xb, qA0 = xa - xb, pA1 = xc + xd, qA1 = xc - xd;
      const F qB0 = xe - xf, qB1 = xg - xh;
      aP0 = S::mfma(t0(lr, t), pA0, aP0);
      aP1 = S::mfma(t0(16 + lr, t), pA0, aP1);
      aP0 = S::mfma(t0(lr, 16 + t), pA1, aP0);
      aP1 = S::mfma(t0(16 + lr, 16 + t), pA1, aP1);
      aMe = S::mfma(t16(0, lr, t), qA0 + qA1, aMe);
      aMo = S::mfma(t16(1, lr, t), qA0 - qA1, aMo);
      bMe = S::mfma(t16(2, lr, t), qB0 + qB1, bMe);
      bMo = S::mfma(t16(3, lr, t), qB0 - qB1, bMo);
      bEv = S::mfma(t16(4, lr, t), xi + xj, bEv);
      bOd = S::mfma(t16(5, lr, t), xk + xl, bOd);
    }
    // a wave reads and writes only its own columns of its own plane
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = S::orow(lk, v);
      const F E0 = bEv[v] + bOd[v], E1 = bEv[v] - bOd[v];
      xp[(2 * q) * XW + col] = aP0[v] + E0;
      xp[(126 - 2 * q) * XW + col] = aP0[v] - E0;
      xp[(62 - 2 * q) * XW + col] = aP1[v] + E1;
      xp[(64 + 2 * q) * XW + col] = aP1[v] - E1;
      xp[(4 * q + 1) * XW + col] = aMe[v] + bMe[v];
      xp[(125 - 4 * q) * XW + col] = aMe[v] - bMe[v];
      xp[(4 * q + 3) * XW + col] = aMo[v] + bMo[v];
      if (q < 15) xp[(123 - 4 * q) * XW + col] = aMo[v] - bMo[v];
    }
  };

  const StripRange sr = xcd_strips(nslab);
  if (sr.first < sr.end) load(sr.first);
  for (int s = sr.first; s < sr.end; s += sr.step) {
    const Slice c = slice(s);
    int lo = lane;
    asm volatile("" : "+v"(lo));
    lr = lo & 15;
    lk = lo >> 4;
    __syncthreads();   // the previous slice's stores have read X (and T, tax are in place)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      F* xp = X[i < 8 ? 0 : 1] + (16 * (i & 7) + rz) * XW;
      xp[2 * cp] = pf[i].x;
      xp[2 * cp + 1] = pf[i].y;
    }
    if (s + sr.step < sr.end) load(s + sr.step);
    __syncthreads();

    // ---- forward product along z
    product();
    __syncthreads();

    // ---- shifted divide: thread -> column tid % 64, rows tid / 64 + 8 i
    {
      const int x = tid & (XW - 1), xg = c.xh * XW + x;
      const bool valid = xg < a.m1;
      const double cst = tmu1[xg] + tmu2[c.y];
      const bool real_pair = a.packed && c.k == 0;
      const double lre = lam[2 * c.k], lim = lam[2 * c.k + 1];
      const double lre1 = real_pair ? lam[2 * a.nk] : 0.0;
      for (int r = tid / XW; r < a.m3; r += 512 / XW) {
        F vr = X[0][r * XW + x], vi = X[1][r * XW + x];
        if (!valid) {
          vr = F(0);
          vi = F(0);
        } else {
          const double mu = cst + tax[r];
          if (real_pair) {
            vr = vr / (F)(lre + mu);
            vi = vi / (F)(lre1 + mu);
          } else {
            const F cc = (F)(lre + mu), dd = (F)lim;
            const F inv = F(1) / (cc * cc + dd * dd);
            const F nr = (vr * cc + vi * dd) * inv;
            const F ni = (vi * cc - vr * dd) * inv;
            vr = nr;
            vi = ni;
          }
        }
        X[0][r * XW + x] = vr;
        X[1][r * XW + x] = vi;
      }
    }
    __syncthreads();

    // ---- inverse product along z, then the slices back in place
    product();
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const F* xp = X[i < 8 ? 0 : 1] + (16 * (i & 7) + rz) * XW;
      F* b = spec + (i < 8 ? c.b0 : c.b1) + (int64_t)(16 * (i & 7) + rz) * zs;
      reinterpret_cast<T2*>(b)[cp] = T2{xp[2 * cp], xp[2 * cp + 1]};
    }
  }
}

}  // namespace

template <typename F, bool L3>
hipError_t launch_xy(F* spec, const F* tab, const SlabArgs& a, hipStream_t s) {
  const int64_t nslab = (int64_t)a.nk * 2 * a.m3;
  if (nslab > 0x7fffffff) return hipErrorInvalidConfiguration;
  static const int resident = persistent_grid(k_dst_xy<F, L3>, 512);
  if (resident < 8) return hipErrorInvalidDeviceFunction;
  hipLaunchKernelGGL((k_dst_xy<F, L3>), dim3(strip_grid(resident, nslab)), dim3(512), 0, s, spec,
                     tab, a);
  return hipGetLastError();
}

template <typename F>
hipError_t launch_dst_xy(F* spec, const F* tab, const SlabArgs& a, hipStream_t s,
                         const F* tab3) {
  if (!spec || !tab || a.nk < 1 || a.m3 < 1 || a.m1 % 2 == 0 || a.m2 % 2 == 0 ||
      a.m1 <= XYP / 2 || a.m1 > XYP || a.m2 <= XYP / 2 || a.m2 > XYP || a.P1 != XYP ||
      a.P2 != XYP || a.P3 < a.m3 || a.PS != (int64_t)a.P1 * a.P2 * a.P3)
    return hipErrorInvalidValue;
  if (tab3 && a.m1 == XYP - 1 && a.m2 == XYP - 1) return launch_xy<F, true>(spec, tab3, a, s);
  return launch_xy<F, false>(spec, tab, a, s);
}

hipError_t launch_dst_zdiv(double* spec, const double* tab3, const SlabArgs& a,
                           const double* lam, const double* tmu1, const double* tmu2,
                           const double* tmu3, hipStream_t s) {
  if (!spec || !tab3 || !lam || !tmu1 || !tmu2 || !tmu3 || a.nk < 1 || a.m3 != XYP - 1 ||
      a.m1 < 1 || a.m1 > XYP || a.m2 < 1 || a.m2 > XYP || a.P1 != XYP || a.P2 != XYP ||
      a.P3 != XYP || a.PS != (int64_t)XYP * XYP * XYP)
    return hipErrorInvalidValue;
  const int64_t nslab = (int64_t)a.nk * a.m2 * 2;
  if (nslab > 0x7fffffff) return hipErrorInvalidConfiguration;
  static const int resident = persistent_grid(k_dst_zdiv<double>, 512);
  if (resident < 8) return hipErrorInvalidDeviceFunction;
  hipLaunchKernelGGL((k_dst_zdiv<double>), dim3(strip_grid(resident, nslab)), dim3(512), 0, s,
                     spec, tab3, a, lam, tmu1, tmu2, tmu3);
  return hipGetLastError();
}

template hipError_t launch_dst_xy<double>(double*, const double*, const SlabArgs&, hipStream_t,
                                          const double*);
template hipError_t launch_dst_xy<float>(float*, const float*, const SlabArgs&, hipStream_t,
                                         const float*);

}  // namespace aao
