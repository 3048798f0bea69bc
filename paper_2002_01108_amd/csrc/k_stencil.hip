// All-at-once matrix-vector product y = L x (Section 2, eq. (allatoncesystem);
// p-step form of eq. (pstepscheme) with M = I):
//   y^k = (r0 I + tau K) x^k + r1 x^{k-1} + r2 x^{k-2},  x^{<1} := 0,
// with coefficient 1 in place of r0 on the first level (a backward-Euler first
// step); backward Euler is (r0, r1, r2) = (1, -1, 0), BDF2 (3/2, -2, 1/2).
// K the 3/5/7-point -Laplacian (constant coefficient), the flux-form
// discretisation of -div(a grad .) with coefficients on cell faces, or (2D, no
// y-face array) a nonsymmetric five-point operator given by four coupling
// planes W, E, S, N per node (upwinded convection-diffusion).
//
// One thread owns one spatial point and walks a chunk of time levels, keeping
// x^{k-1} (and x^{k-2}) in registers, so x is read from HBM once per chunk
// (plus one or two halo slabs per chunk) and y written once: 16 B per unknown.  A block is a
// 64 x 4 patch of the x-y plane; spatial neighbours come through L1/L2.
// Workgroups are renumbered so that patches adjacent in y land on the same
// XCD (consecutive hardware workgroup ids rotate over the 8 XCDs).
#include "common.h"

namespace aao {
namespace {

constexpr int TX = 64;       // points along x per block
constexpr int TY = 4;        // rows along y per block
constexpr int TCHUNK = 8;    // time levels per block

// TWO: the scheme has an x^{k-2} term (r2 != 0); backward Euler compiles without it.
template <int DIM, bool VAR, bool TWO>
__global__ __launch_bounds__(TX * TY) void k_apply_L(
    const double* __restrict__ x, double* __restrict__ y, int n, int m1, int m2, int m3,
    int nbx, int nby, int nbt, double c1, double c2, double c3, const double* __restrict__ ax,
    const double* __restrict__ ay, const double* __restrict__ az, double r0, double r1,
    double r2) {
  const int nblk = nbx * nby * m3 * nbt;
  const int b = xcd_remap(blockIdx.x, nblk);
  // logical tile order: x tiles fastest, then y tiles, then z, then time chunk
  int t = b;
  const int bx = t % nbx; t /= nbx;
  const int by = t % nby; t /= nby;
  const int i3 = t % m3;  t /= m3;
  const int bt = t;
  const int i1 = bx * TX + threadIdx.x;
  const int i2 = by * TY + threadIdx.y;
  if (i1 >= m1 || i2 >= m2) return;
  const int64_t m = (int64_t)m1 * m2 * m3;
  const int64_t s = i1 + (int64_t)m1 * (i2 + (int64_t)m2 * i3);
  const int64_t sx = 1, sy = m1, sz = (int64_t)m1 * m2;

  // stencil weights (already multiplied by tau/h^2)
  double wxm, wxp, wym = 0, wyp = 0, wzm = 0, wzp = 0, diag;
  if (VAR) {
    const int64_t fx = (int64_t)(i3 * m2 + i2) * (m1 + 1) + i1;
    wxm = ax[fx];
    wxp = ax[fx + 1];
    diag = 1.0 + wxm + wxp;
    if (DIM >= 2) {
      const int64_t fy = (int64_t)(i3 * (m2 + 1) + i2) * m1 + i1;
      wym = ay[fy];
      wyp = ay[fy + m1];
      diag += wym + wyp;
    }
    if (DIM >= 3) {
      const int64_t fz = (int64_t)(i3 * m2 + i2) * m1 + i1;
      wzm = az[fz];
      wzp = az[fz + (int64_t)m2 * m1];
      diag += wzm + wzp;
    }
  } else {
    wxm = wxp = c1;
    diag = 1.0 + 2.0 * c1;
    if (DIM >= 2) { wym = wyp = c2; diag += 2.0 * c2; }
    if (DIM >= 3) { wzm = wzp = c3; diag += 2.0 * c3; }
  }
  // Dirichlet zero: drop couplings that leave the grid
  const bool hxm = i1 > 0, hxp = i1 < m1 - 1;
  const bool hym = DIM >= 2 && i2 > 0, hyp = DIM >= 2 && i2 < m2 - 1;
  const bool hzm = DIM >= 3 && i3 > 0, hzp = DIM >= 3 && i3 < m3 - 1;

  const int k0 = bt * TCHUNK;
  const int k1 = min(n, k0 + TCHUNK);
  const double dr = r0 - 1.0;   // diag carries 1 (first level); later levels add r0 - 1
  double prev = (k0 > 0) ? x[(int64_t)(k0 - 1) * m + s] : 0.0;
  double prev2 = (TWO && k0 > 1) ? x[(int64_t)(k0 - 2) * m + s] : 0.0;
  for (int k = k0; k < k1; ++k) {
    const double* xk = x + (int64_t)k * m + s;
    const double xc = xk[0];
    double nb = 0.0;
    if (hxm) nb += wxm * xk[-sx];
    if (hxp) nb += wxp * xk[sx];
    if (DIM >= 2) {
      if (hym) nb += wym * xk[-sy];
      if (hyp) nb += wyp * xk[sy];
    }
    if (DIM >= 3) {
      if (hzm) nb += wzm * xk[-sz];
      if (hzp) nb += wzp * xk[sz];
    }
    double v = (k == 0 ? diag : diag + dr) * xc - nb + r1 * prev;
    if (TWO) v += r2 * prev2;
    y[(int64_t)k * m + s] = v;
    prev2 = prev;
    prev = xc;
  }
}

// 2.5D-blocked variant for 2D/3D grids.  A wave owns 64 consecutive x points
// (62 outputs; lanes 0 and 63 carry the x halo) and TY consecutive rows, and
// walks TC time levels: per level it issues the TY+2 row loads at once, takes
// x neighbours from adjacent lanes, y neighbours from its register window and
// x^{k-1} from registers.  Four waves stack in y.
constexpr int XW = 62;

// EPI selects what the block does with L x besides (or instead of) storing it:
//   0: y = L x;
//   1: no store; partial sum of (f - L x)^2 per block into part[blockIdx.x]
//      (the explicit residual norm of a solve, without a residual array);
//   2: y = L x and the partial dot products of y with Q (<= 4) basis vectors
//      into part[blockIdx.x * Q + i] (the first Gram-Schmidt projection of an
//      Arnoldi step, without re-reading y).
struct StencilEpi {
  const double* f;        // EPI 1
  const double* w[4];     // EPI 2: basis vectors
  double* part;
  double* wsq;            // EPI 2, optional: partial sums of (L x)^2 per block
  double* w0sq;           // EPI 2 with Q = 1, optional: partial sums of w[0]^2 per block
};

// Q1: 2D finite elements on a uniform grid (Section 5): L = R (x) M + tau I (x) K with
// M = M1 (x) M1 and K = M1 (x) K1 + K1 (x) M1, both 9-point:
//   M x = qm0 c + qm1 (edge neighbours) + qm2 (corner neighbours)
//   tau K x = qk0 c + qk1 (all eight neighbours)
// with (qm0, qm1, qm2) = h^2/36 (16, 4, 1) and (qk0, qk1) = tau/3 (8, -1).  The
// time terms act on M x, so the wave keeps M x^{k-1} (and M x^{k-2}) and starts
// its chunk one or two levels early to form them.
struct Q1W {
  double m0, m1, m2, k0, k1;
};

template <int DIM, bool VAR, int TY, int TC, int EPI, int Q, bool TWO, bool FE = false,
          bool SQ = false>
__global__ __launch_bounds__(256) void k_apply_L25(
    const double* __restrict__ x, double* __restrict__ y, int n, int m1, int m2, int m3, int nxt,
    int nyt, int nct, double c1, double c2, double c3, const double* __restrict__ ax,
    const double* __restrict__ ay, const double* __restrict__ az, StencilEpi ep, double r0,
    double r1, double r2, Q1W qw) {
  static_assert(!FE || (DIM == 2 && !VAR), "Q1 elements: 2D, constant coefficient");
  const int nblk = nxt * nyt * m3 * nct;
  int b = xcd_remap(blockIdx.x, nblk);
  const int bx = b % nxt; b /= nxt;
  const int by = b % nyt; b /= nyt;
  const int i3 = b % m3;
  const int bc = b / m3;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i1 = bx * XW - 1 + lane;
  const bool inx = i1 >= 0 && i1 < m1;
  const bool writer = lane >= 1 && lane <= XW && inx;
  const int j0 = (by * 4 + wave) * TY;
  // a wave past the last row has nothing to do, but stays for the block reduction
  const bool wave_on = j0 < m2;
  constexpr int NQ = EPI == 2 ? Q : 1;
  // EPI 2 also sums (L x)^2 and (SQ, one basis vector) that vector's squares
  constexpr bool SQ0 = SQ && EPI == 2 && Q == 1;
  constexpr int NR = EPI == 2 ? Q + 1 + (SQ0 ? 1 : 0) : 1;
  double red_acc[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) red_acc[i] = 0.0;
  const int64_t m = (int64_t)m1 * m2 * m3;
  const int64_t pl = (int64_t)m1 * m2;
  const int64_t base = (int64_t)i3 * pl + i1;

  // per-row weights (constant over time) and diagonal
  double wxm[TY], wxp[TY], wym[TY], wyp[TY], wzm[TY], wzp[TY], dg[TY];
#pragma unroll
  for (int t = 0; t < TY; ++t) {
    const int j = j0 + t;
    const bool ok = inx && j < m2;
    if (VAR && DIM == 2 && ay == nullptr) {   // coupling planes [W, E, S, N][m2][m1]
      const int64_t p = (int64_t)j * m1 + i1;
      wxm[t] = ok ? ax[p] : 0.0;
      wxp[t] = ok ? ax[p + pl] : 0.0;
      wym[t] = ok ? ax[p + 2 * pl] : 0.0;
      wyp[t] = ok ? ax[p + 3 * pl] : 0.0;
      wzm[t] = wzp[t] = 0.0;
    } else if (VAR) {
      const int64_t fx = ((int64_t)i3 * m2 + j) * (m1 + 1) + i1;
      const int64_t fy = ((int64_t)i3 * (m2 + 1) + j) * m1 + i1;
      wxm[t] = ok ? ax[fx] : 0.0;
      wxp[t] = ok ? ax[fx + 1] : 0.0;
      wym[t] = ok ? ay[fy] : 0.0;
      wyp[t] = ok ? ay[fy + m1] : 0.0;
      if (DIM >= 3) {
        const int64_t fz = ((int64_t)i3 * m2 + j) * m1 + i1;
        wzm[t] = ok ? az[fz] : 0.0;
        wzp[t] = ok ? az[fz + pl] : 0.0;
      } else {
        wzm[t] = wzp[t] = 0.0;
      }
    } else {
      wxm[t] = wxp[t] = c1;
      wym[t] = wyp[t] = c2;
      wzm[t] = wzp[t] = (DIM >= 3) ? c3 : 0.0;
    }
    dg[t] = 1.0 + wxm[t] + wxp[t] + wym[t] + wyp[t] + wzm[t] + wzp[t];
  }
  const bool zlo = DIM >= 3 && i3 > 0, zhi = DIM >= 3 && i3 < m3 - 1;

  const int k0 = bc * TC;
  const int k1 = wave_on ? min(n, k0 + TC) : k0;
  const double dr = r0 - 1.0;   // dg carries 1 (first level); later levels add r0 - 1
  // prev / prev2: x^{k-1} / x^{k-2} (finite differences), M x^{k-1} / M x^{k-2} (Q1)
  double prev[TY], prev2[TWO ? TY : 1];
#pragma unroll
  for (int t = 0; t < TY; ++t) {
    const int j = j0 + t;
    prev[t] = (!FE && k0 > 0 && inx && j < m2)
                  ? x[(int64_t)(k0 - 1) * m + base + (int64_t)j * m1] : 0.0;
    if (TWO)
      prev2[TWO ? t : 0] = (!FE && k0 > 1 && inx && j < m2)
                               ? x[(int64_t)(k0 - 2) * m + base + (int64_t)j * m1] : 0.0;
  }
  // Q1: run the levels before the chunk (at most 1 + TWO, not below level 0)
  // without output, to form M x^{k0-1} and M x^{k0-2}
  const int kstart = FE ? max(0, k0 - (TWO ? 2 : 1)) : k0;
  for (int k = (wave_on ? kstart : k1); k < k1; ++k) {
    const double* xk = x + (int64_t)k * m + base;
    double r[TY + 2];
#pragma unroll
    for (int t = 0; t < TY + 2; ++t) {
      const int j = j0 - 1 + t;
      r[t] = (inx && j >= 0 && j < m2) ? xk[(int64_t)j * m1] : 0.0;
    }
    double zl[TY], zh[TY];
#pragma unroll
    for (int t = 0; t < TY; ++t) {
      const int j = j0 + t;
      const bool ok = inx && j < m2;
      zl[t] = (ok && zlo) ? xk[(int64_t)j * m1 - pl] : 0.0;
      zh[t] = (ok && zhi) ? xk[(int64_t)j * m1 + pl] : 0.0;
    }
    // epilogue operands are loaded together with the rows so their latency overlaps
    double eo[NQ][TY];
    if (EPI != 0) {
#pragma unroll
      for (int t = 0; t < TY; ++t) {
        const bool ok = writer && j0 + t < m2 && (!FE || k >= k0);
        const int64_t off = (int64_t)k * m + base + (int64_t)(j0 + t) * m1;
#pragma unroll
        for (int i = 0; i < NQ; ++i) eo[i][t] = ok ? (EPI == 1 ? ep.f : ep.w[i])[off] : 0.0;
      }
    }
    double* yk = y + (int64_t)k * m + base;
#pragma unroll
    for (int t = 0; t < TY; ++t) {
      const double c = r[t + 1];
      const double left = __shfl_up(c, 1, 64);
      const double right = __shfl_down(c, 1, 64);
      double acc, mx = 0.0;
      if (FE) {
        const double se = left + right + r[t] + r[t + 2];
        const double sc = __shfl_up(r[t], 1, 64) + __shfl_down(r[t], 1, 64) +
                          __shfl_up(r[t + 2], 1, 64) + __shfl_down(r[t + 2], 1, 64);
        mx = qw.m0 * c + qw.m1 * se + qw.m2 * sc;
        acc = (k == 0 ? mx : r0 * mx) + (qw.k0 * c + qw.k1 * (se + sc)) + r1 * prev[t];
      } else {
        acc = (k == 0 ? dg[t] : dg[t] + dr) * c - wxm[t] * left - wxp[t] * right -
              wym[t] * r[t] - wyp[t] * r[t + 2] + r1 * prev[t];
      }
      if (TWO) acc += r2 * prev2[TWO ? t : 0];
      if (DIM >= 3) acc -= wzm[t] * zl[t] + wzp[t] * zh[t];
      if (FE && k < k0) {   // a level before the chunk: history only
        if (TWO) prev2[TWO ? t : 0] = prev[t];
        prev[t] = mx;
        continue;
      }
      const bool out_ok = writer && j0 + t < m2;
      if (EPI != 1 && out_ok && y) yk[(int64_t)(j0 + t) * m1] = acc;
      if (EPI == 1 && out_ok) {
        const double d = eo[0][t] - acc;
        red_acc[0] += d * d;
      }
      if (EPI == 2 && out_ok) {
#pragma unroll
        for (int i = 0; i < NQ; ++i) red_acc[i] += eo[i][t] * acc;
        red_acc[NQ] += acc * acc;
        if (SQ0) red_acc[NR - 1] += eo[0][t] * eo[0][t];
      }
      if (TWO) prev2[TWO ? t : 0] = prev[t];
      prev[t] = FE ? mx : c;
    }
  }
  if (EPI != 0) {
    // block reduction: wave sums, then one value per output from LDS
    __shared__ double red[NR][4];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      double v = red_acc[i];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0) red[i][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < NR) {
      const double v =
          red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
      if (threadIdx.x < NQ)
        ep.part[(int64_t)blockIdx.x * NQ + threadIdx.x] = v;
      else if (threadIdx.x == NQ && ep.wsq)
        ep.wsq[blockIdx.x] = v;
      else if (SQ0 && threadIdx.x == NQ + 1 && ep.w0sq)
        ep.w0sq[blockIdx.x] = v;
    }
  }
}

// 3D z-marching variant.  The 2.5D walk above reads the planes z-1 and z+1 of
// every output plane again (three reads of each plane, of which the caches
// catch about half).  Here a block owns a 62 x (4 TYZ) patch of the x-y plane,
// a range of ZBZ planes and TCZ time levels, and walks up in z keeping, for
// each of its time levels, the planes z-1 (its own rows), z and z+1 (with the
// y-halo rows) in registers: each plane is loaded once per block, and x^{k-1}
// comes from the window of the previous level except at the first level of
// the chunk.  Epilogues as in k_apply_L25.  The window costs TCZ (3 TYZ + 4)
// doubles per lane; of the shapes measured at 127^3 x 256 (TYZ 2..8, TCZ 2..4,
// ZBZ 32..128) TYZ = 4, TCZ = 2, ZBZ = 32 was fastest: 2.52 ms for L v against
// 2.85 ms for the 2.5D walk.
constexpr int TYZ = 4, TCZ = 2, ZBZ = 32;
// Time chunks are ordered in groups of CGZ just inside the x tiles, so that
// the chunks of one patch that follow each other in time run at the same time
// on one XCD: the level before a chunk, which the previous chunk of the group
// loads as its own, then usually comes from L2 (when the chunk count allows it).
constexpr int CGZ = 4;

template <bool VAR, int EPI, int Q, bool TWO, bool SQ = false>
__global__ __launch_bounds__(256) void k_apply_L3z(
    const double* __restrict__ x, double* __restrict__ y, int n, int m1, int m2, int m3, int nxt,
    int nyt, int nzt, int nct, double c1, double c2, double c3, const double* __restrict__ ax,
    const double* __restrict__ ay, const double* __restrict__ az, StencilEpi ep, double r0,
    double r1, double r2) {
  constexpr int TY = TYZ, TC = TCZ;
  const int nblk = nxt * nyt * nzt * nct;
  int b = xcd_remap(blockIdx.x, nblk);
  const int cg = nct % CGZ == 0 ? CGZ : 1;
  const int bx = b % nxt; b /= nxt;
  const int cl = b % cg; b /= cg;
  const int by = b % nyt; b /= nyt;
  const int bz = b % nzt;
  const int bc = (b / nzt) * cg + cl;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i1 = bx * XW - 1 + lane;
  const bool inx = i1 >= 0 && i1 < m1;
  const bool writer = lane >= 1 && lane <= XW && inx;
  const int j0 = (by * 4 + wave) * TY;
  const int k0 = bc * TC;
  // levels of this chunk (a wave past the last row has none, but stays for the
  // block reduction)
  const int kn = j0 < m2 ? min(n, k0 + TC) - k0 : 0;
  const int z0 = bz * ZBZ, z1 = min(m3, z0 + ZBZ);
  constexpr int NQ = EPI == 2 ? Q : 1;
  // EPI 2 also sums (L x)^2 and (SQ, one basis vector) that vector's squares
  constexpr bool SQ0 = SQ && EPI == 2 && Q == 1;
  constexpr int NR = EPI == 2 ? Q + 1 + (SQ0 ? 1 : 0) : 1;
  double red_acc[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) red_acc[i] = 0.0;
  const int64_t m = (int64_t)m1 * m2 * m3;
  const int64_t pl = (int64_t)m1 * m2;
  const double dr = r0 - 1.0;   // the diagonal carries 1 (first level); later levels add r0 - 1

  // rows j0 - 1 + t (t < TY + 2) of plane z at level k0 + kk; zero outside the grid
  auto load_ext = [&](int kk, int z, double* dst) {
    const bool zok = kk < kn && z >= 0 && z < m3 && inx;
    const double* src = x + (int64_t)(k0 + kk) * m + (int64_t)z * pl + i1;
#pragma unroll
    for (int t = 0; t < TY + 2; ++t) {
      const int j = j0 - 1 + t;
      dst[t] = (zok && j >= 0 && j < m2) ? src[(int64_t)j * m1] : 0.0;
    }
  };
  // rows j0 + t (t < TY) of plane z at level k (k may be before the chunk)
  auto load_own = [&](int k, int z, double* dst) {
    const bool ok = kn > 0 && k >= 0 && z >= 0 && z < m3 && inx;
    const double* src = x + (int64_t)k * m + (int64_t)z * pl + i1;
#pragma unroll
    for (int t = 0; t < TY; ++t) {
      const int j = j0 + t;
      dst[t] = (ok && j < m2) ? src[(int64_t)j * m1] : 0.0;
    }
  };

  double lo[TC][TY], ce[TC][TY + 2], hi[TC][TY + 2];
#pragma unroll
  for (int kk = 0; kk < TC; ++kk) {
    load_own(kk < kn ? k0 + kk : -1, z0 - 1, lo[kk]);
    load_ext(kk, z0, ce[kk]);
    load_ext(kk, z0 + 1, hi[kk]);
  }
  for (int z = kn > 0 ? z0 : z1; z < z1; ++z) {
    // the chunk's history at plane z: x^{k0-1} (and x^{k0-2})
    double hp[TY], hp2[TWO ? TY : 1];
    load_own(k0 - 1, z, hp);
    if (TWO) load_own(k0 - 2, z, hp2);
    // per-row weights at plane z (already multiplied by tau/h^2) and diagonal
    double wxm[TY], wxp[TY], wym[TY], wyp[TY], wzm[TY], wzp[TY], dg[TY];
#pragma unroll
    for (int t = 0; t < TY; ++t) {
      const int j = j0 + t;
      if (VAR) {
        const bool ok = inx && j < m2;
        const int64_t fx = ((int64_t)z * m2 + j) * (m1 + 1) + i1;
        const int64_t fy = ((int64_t)z * (m2 + 1) + j) * m1 + i1;
        const int64_t fz = ((int64_t)z * m2 + j) * m1 + i1;
        wxm[t] = ok ? ax[fx] : 0.0;
        wxp[t] = ok ? ax[fx + 1] : 0.0;
        wym[t] = ok ? ay[fy] : 0.0;
        wyp[t] = ok ? ay[fy + m1] : 0.0;
        wzm[t] = ok ? az[fz] : 0.0;
        wzp[t] = ok ? az[fz + pl] : 0.0;
      } else {
        wxm[t] = wxp[t] = c1;
        wym[t] = wyp[t] = c2;
        wzm[t] = wzp[t] = c3;
      }
      dg[t] = 1.0 + wxm[t] + wxp[t] + wym[t] + wyp[t] + wzm[t] + wzp[t];
    }
#pragma unroll
    for (int kk = 0; kk < TC; ++kk) {
      if (kk >= kn) break;
      const int k = k0 + kk;
      const int64_t rowoff = (int64_t)k * m + (int64_t)z * pl + i1;
      double eo[NQ][TY];
      if (EPI != 0) {
#pragma unroll
        for (int t = 0; t < TY; ++t) {
          const bool ok = writer && j0 + t < m2;
          const int64_t off = rowoff + (int64_t)(j0 + t) * m1;
#pragma unroll
          for (int i = 0; i < NQ; ++i) eo[i][t] = ok ? (EPI == 1 ? ep.f : ep.w[i])[off] : 0.0;
        }
      }
#pragma unroll
      for (int t = 0; t < TY; ++t) {
        const double c = ce[kk][t + 1];
        const double left = __shfl_up(c, 1, 64);
        const double right = __shfl_down(c, 1, 64);
        const double pv = kk == 0 ? hp[t] : ce[kk > 0 ? kk - 1 : 0][t + 1];
        double acc = (k == 0 ? dg[t] : dg[t] + dr) * c - wxm[t] * left - wxp[t] * right -
                     wym[t] * ce[kk][t] - wyp[t] * ce[kk][t + 2] - wzm[t] * lo[kk][t] -
                     wzp[t] * hi[kk][t + 1] + r1 * pv;
        if (TWO) {
          const double pv2 =
              kk == 0 ? hp2[TWO ? t : 0] : (kk == 1 ? hp[t] : ce[kk > 1 ? kk - 2 : 0][t + 1]);
          acc += r2 * pv2;
        }
        const bool out_ok = writer && j0 + t < m2;
        if (EPI != 1 && out_ok && y) y[rowoff + (int64_t)(j0 + t) * m1] = acc;
        if (EPI == 1 && out_ok) {
          const double d = eo[0][t] - acc;
          red_acc[0] += d * d;
        }
        if (EPI == 2 && out_ok) {
#pragma unroll
          for (int i = 0; i < NQ; ++i) red_acc[i] += eo[i][t] * acc;
          red_acc[NQ] += acc * acc;
          if (SQ0) red_acc[NR - 1] += eo[0][t] * eo[0][t];
        }
      }
    }
    // advance the windows one plane up
    if (z + 1 < z1) {
#pragma unroll
      for (int kk = 0; kk < TC; ++kk) {
#pragma unroll
        for (int t = 0; t < TY; ++t) lo[kk][t] = ce[kk][t + 1];
#pragma unroll
        for (int t = 0; t < TY + 2; ++t) ce[kk][t] = hi[kk][t];
        load_ext(kk, z + 2, hi[kk]);
      }
    }
  }
  if (EPI != 0) {
    __shared__ double red[NR][4];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      double v = red_acc[i];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0) red[i][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < NR) {
      const double v =
          red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
      if (threadIdx.x < NQ)
        ep.part[(int64_t)blockIdx.x * NQ + threadIdx.x] = v;
      else if (threadIdx.x == NQ && ep.wsq)
        ep.wsq[blockIdx.x] = v;
      else if (SQ0 && threadIdx.x == NQ + 1 && ep.w0sq)
        ep.w0sq[blockIdx.x] = v;
    }
  }
}

constexpr int TY25 = 8, TC25 = 8;

// block counts of the 3D z-marching walk
struct Grid3z {
  int nxt, nyt, nzt, nct;
  int64_t blocks() const { return (int64_t)nxt * nyt * nzt * nct; }
};
Grid3z grid3z(const Geometry& g) {
  return {(g.m1 + XW - 1) / XW, (g.m2 + 4 * TYZ - 1) / (4 * TYZ), (g.m3 + ZBZ - 1) / ZBZ,
          (g.n + TCZ - 1) / TCZ};
}
bool use3z(const Geometry& g) { return g.dim == 3 && !g.q1; }

int64_t blocks25(const Geometry& g) {
  if (use3z(g)) return grid3z(g).blocks();
  const int nxt = (g.m1 + XW - 1) / XW;
  const int nyt = (g.m2 + 4 * TY25 - 1) / (4 * TY25);
  const int nct = (g.n + TC25 - 1) / TC25;
  return (int64_t)nxt * nyt * g.m3 * nct;
}

template <int DIM, bool VAR, int EPI, int Q = 1>
hipError_t launch25(const Geometry& g, const double* x, double* y, double c1, double c2,
                    double c3, const double* ax, const double* ay, const double* az,
                    const StencilEpi& ep, hipStream_t s) {
  const bool two = g.r2 != 0.0;
  const Q1W qw{g.qm[0], g.qm[1], g.qm[2], g.qk[0], g.qk[1]};
  const int nxt = (g.m1 + XW - 1) / XW;
  const int nyt = (g.m2 + 4 * TY25 - 1) / (4 * TY25);
  const int nct = (g.n + TC25 - 1) / TC25;
  const int64_t nblk = blocks25(g);
  if (nblk <= 0 || nblk > 0x7fffffff) return hipErrorInvalidConfiguration;
  // the variants that also sum the basis vector's squares exist for one basis
  // vector only and run only when asked for (their extra accumulator costs the
  // 2D kernel a wave per SIMD)
  constexpr bool SQOK = EPI == 2 && Q == 1;
  const bool sq = ep.w0sq != nullptr;
  if (sq && !SQOK) return hipErrorInvalidValue;
  if constexpr (DIM == 3) {
    if (use3z(g)) {
      const Grid3z gz = grid3z(g);
#define L3Z_LAUNCH(TW, S)                                                                     \
  hipLaunchKernelGGL((k_apply_L3z<VAR, EPI, Q, TW, S>), dim3((unsigned)nblk), dim3(256), 0, s, \
                     x, y, g.n, g.m1, g.m2, g.m3, gz.nxt, gz.nyt, gz.nzt, gz.nct, c1, c2, c3, ax, \
                     ay, az, ep, g.r0, g.r1, g.r2)
      if (sq) {
        if constexpr (SQOK) {
          if (two) L3Z_LAUNCH(true, true);
          else L3Z_LAUNCH(false, true);
        }
      } else if (two) {
        L3Z_LAUNCH(true, false);
      } else {
        L3Z_LAUNCH(false, false);
      }
#undef L3Z_LAUNCH
      return hipGetLastError();
    }
  }
#define L25_LAUNCH(TW, F, S)                                                                   \
  hipLaunchKernelGGL((k_apply_L25<DIM, VAR, TY25, TC25, EPI, Q, TW, F, S>),                     \
                     dim3((unsigned)nblk), dim3(256), 0, s, x, y, g.n, g.m1, g.m2, g.m3, nxt, nyt, \
                     nct, c1, c2, c3, ax, ay, az, ep, g.r0, g.r1, g.r2, qw)
  if (sq) {
    if constexpr (SQOK) {
      if (g.q1) {
        if constexpr (DIM == 2 && !VAR) {
          if (two) L25_LAUNCH(true, true, true);
          else L25_LAUNCH(false, true, true);
        } else {
          return hipErrorInvalidValue;
        }
      } else if (two) {
        L25_LAUNCH(true, false, true);
      } else {
        L25_LAUNCH(false, false, true);
      }
    }
  } else if (g.q1) {
    if constexpr (DIM == 2 && !VAR) {
      if (two) L25_LAUNCH(true, true, false);
      else L25_LAUNCH(false, true, false);
    } else {
      return hipErrorInvalidValue;   // Q1 elements: 2D constant coefficient only
    }
  } else if (two) {
    L25_LAUNCH(true, false, false);
  } else {
    L25_LAUNCH(false, false, false);
  }
#undef L25_LAUNCH
  return hipGetLastError();
}

template <int DIM, bool VAR>
hipError_t launch(const Geometry& g, const double* x, double* y, double c1, double c2, double c3,
                  const double* ax, const double* ay, const double* az, hipStream_t s) {
  if (DIM >= 2) return launch25<DIM, VAR, 0>(g, x, y, c1, c2, c3, ax, ay, az, StencilEpi{}, s);
  const int nbx = (g.m1 + TX - 1) / TX;
  const int nby = (g.m2 + TY - 1) / TY;
  const int nbt = (g.n + TCHUNK - 1) / TCHUNK;
  const int64_t nblk = (int64_t)nbx * nby * g.m3 * nbt;
  if (nblk <= 0 || nblk > 0x7fffffff) return hipErrorInvalidConfiguration;
  if (g.r2 != 0.0)
    hipLaunchKernelGGL((k_apply_L<DIM, VAR, true>), dim3((unsigned)nblk), dim3(TX, TY), 0, s, x,
                       y, g.n, g.m1, g.m2, g.m3, nbx, nby, nbt, c1, c2, c3, ax, ay, az, g.r0,
                       g.r1, g.r2);
  else
    hipLaunchKernelGGL((k_apply_L<DIM, VAR, false>), dim3((unsigned)nblk), dim3(TX, TY), 0, s, x,
                       y, g.n, g.m1, g.m2, g.m3, nbx, nby, nbt, c1, c2, c3, ax, ay, az, g.r0,
                       g.r1, g.r2);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_apply_L(const Geometry& g, const double* x, double* y, double c1, double c2,
                          double c3, hipStream_t s) {
  switch (g.dim) {
    case 1: return launch<1, false>(g, x, y, c1, c2, c3, nullptr, nullptr, nullptr, s);
    case 2: return launch<2, false>(g, x, y, c1, c2, c3, nullptr, nullptr, nullptr, s);
    case 3: return launch<3, false>(g, x, y, c1, c2, c3, nullptr, nullptr, nullptr, s);
  }
  return hipErrorInvalidValue;
}

int64_t stencil_partials(const Geometry& g) { return g.dim >= 2 ? blocks25(g) : 0; }

hipError_t launch_apply_L_epi(const Geometry& g, int epi, const double* x, double* y,
                              const double* f, const double* const* basis, int q, double* part,
                              double* wsq, double* w0sq, double c1, double c2, double c3,
                              const double* ax, const double* ay, const double* az,
                              hipStream_t s) {
  if (g.dim < 2 || (epi == 2 && (q < 1 || q > kStencilDotsMax)) || (epi != 1 && epi != 2))
    return hipErrorInvalidValue;
  if (w0sq && !(epi == 2 && q == 1)) return hipErrorInvalidValue;
  StencilEpi ep{};
  ep.f = f;
  for (int i = 0; i < 4; ++i) ep.w[i] = (epi == 2 && i < q) ? basis[i] : nullptr;
  ep.part = part;
  ep.wsq = epi == 2 ? wsq : nullptr;
  ep.w0sq = w0sq;
  const bool var = ax != nullptr;
#define L25(D, V, E, Q) launch25<D, V, E, Q>(g, x, y, c1, c2, c3, ax, ay, az, ep, s)
#define DOTS(D, V)                        \
  switch (q) {                            \
    case 1: return L25(D, V, 2, 1);       \
    case 2: return L25(D, V, 2, 2);       \
    case 3: return L25(D, V, 2, 3);       \
    default: return L25(D, V, 2, 4);      \
  }
  if (g.dim == 2) {
    if (epi == 1) return var ? L25(2, true, 1, 1) : L25(2, false, 1, 1);
    if (var) { DOTS(2, true) }
    DOTS(2, false)
  }
  if (epi == 1) return var ? L25(3, true, 1, 1) : L25(3, false, 1, 1);
  if (var) { DOTS(3, true) }
  DOTS(3, false)
#undef DOTS
#undef L25
}

hipError_t launch_apply_L_var(const Geometry& g, const double* x, double* y, const double* ax,
                              const double* ay, const double* az, hipStream_t s) {
  switch (g.dim) {
    case 1: return launch<1, true>(g, x, y, 0, 0, 0, ax, ay, az, s);
    case 2: return launch<2, true>(g, x, y, 0, 0, 0, ax, ay, az, s);
    case 3: return launch<3, true>(g, x, y, 0, 0, 0, ax, ay, az, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace aao
