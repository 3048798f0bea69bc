// All-at-once matrix-vector product y = L x (Section 2, eq. (allatoncesystem)):
//   y^k = (I + tau K) x^k - x^{k-1},  x^0 := 0,
// K the 3/5/7-point -Laplacian (constant coefficient) or the flux-form
// discretisation of -div(a grad .) with coefficients on cell faces.
//
// One thread owns one spatial point and walks a chunk of time levels, keeping
// x^{k-1} in a register, so x is read from HBM once per chunk (plus one
// halo slab per chunk) and y written once: 16 B per unknown.  A block is a
// 64 x 4 patch of the x-y plane; spatial neighbours come through L1/L2.
// Workgroups are renumbered so that patches adjacent in y land on the same
// XCD (consecutive hardware workgroup ids rotate over the 8 XCDs).
#include "common.h"

namespace aao {
namespace {

constexpr int TX = 64;       // points along x per block
constexpr int TY = 4;        // rows along y per block
constexpr int TCHUNK = 8;    // time levels per block

template <int DIM, bool VAR>
__global__ __launch_bounds__(TX * TY) void k_apply_L(
    const double* __restrict__ x, double* __restrict__ y, int n, int m1, int m2, int m3,
    int nbx, int nby, int nbt, double c1, double c2, double c3, const double* __restrict__ ax,
    const double* __restrict__ ay, const double* __restrict__ az) {
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
  double prev = (k0 > 0) ? x[(int64_t)(k0 - 1) * m + s] : 0.0;
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
    y[(int64_t)k * m + s] = diag * xc - nb - prev;
    prev = xc;
  }
}

// 2.5D-blocked variant for 2D/3D grids.  A wave owns 64 consecutive x points
// (62 outputs; lanes 0 and 63 carry the x halo) and TY consecutive rows, and
// walks TC time levels: per level it issues the TY+2 row loads at once, takes
// x neighbours from adjacent lanes, y neighbours from its register window and
// x^{k-1} from registers.  Four waves stack in y.
constexpr int XW = 62;

template <int DIM, bool VAR, int TY, int TC>
__global__ __launch_bounds__(256) void k_apply_L25(
    const double* __restrict__ x, double* __restrict__ y, int n, int m1, int m2, int m3, int nxt,
    int nyt, int nct, double c1, double c2, double c3, const double* __restrict__ ax,
    const double* __restrict__ ay, const double* __restrict__ az) {
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
  if (j0 >= m2) return;
  const int64_t m = (int64_t)m1 * m2 * m3;
  const int64_t pl = (int64_t)m1 * m2;
  const int64_t base = (int64_t)i3 * pl + i1;

  // per-row weights (constant over time) and diagonal
  double wxm[TY], wxp[TY], wym[TY], wyp[TY], wzm[TY], wzp[TY], dg[TY];
#pragma unroll
  for (int t = 0; t < TY; ++t) {
    const int j = j0 + t;
    const bool ok = inx && j < m2;
    if (VAR) {
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
  const int k1 = min(n, k0 + TC);
  double prev[TY];
#pragma unroll
  for (int t = 0; t < TY; ++t) {
    const int j = j0 + t;
    prev[t] = (k0 > 0 && inx && j < m2) ? x[(int64_t)(k0 - 1) * m + base + (int64_t)j * m1] : 0.0;
  }
  for (int k = k0; k < k1; ++k) {
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
    double* yk = y + (int64_t)k * m + base;
#pragma unroll
    for (int t = 0; t < TY; ++t) {
      const double c = r[t + 1];
      const double left = __shfl_up(c, 1, 64);
      const double right = __shfl_down(c, 1, 64);
      double acc = dg[t] * c - wxm[t] * left - wxp[t] * right - wym[t] * r[t] -
                   wyp[t] * r[t + 2] - prev[t];
      if (DIM >= 3) acc -= wzm[t] * zl[t] + wzp[t] * zh[t];
      if (writer && j0 + t < m2) yk[(int64_t)(j0 + t) * m1] = acc;
      prev[t] = c;
    }
  }
}

template <int DIM, bool VAR>
hipError_t launch25(const Geometry& g, const double* x, double* y, double c1, double c2,
                    double c3, const double* ax, const double* ay, const double* az,
                    hipStream_t s) {
  constexpr int TY = 8, TC = 8;
  const int nxt = (g.m1 + XW - 1) / XW;
  const int nyt = (g.m2 + 4 * TY - 1) / (4 * TY);
  const int nct = (g.n + TC - 1) / TC;
  const int64_t nblk = (int64_t)nxt * nyt * g.m3 * nct;
  if (nblk <= 0 || nblk > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_apply_L25<DIM, VAR, TY, TC>), dim3((unsigned)nblk), dim3(256), 0, s, x, y,
                     g.n, g.m1, g.m2, g.m3, nxt, nyt, nct, c1, c2, c3, ax, ay, az);
  return hipGetLastError();
}

template <int DIM, bool VAR>
hipError_t launch(const Geometry& g, const double* x, double* y, double c1, double c2, double c3,
                  const double* ax, const double* ay, const double* az, hipStream_t s) {
  if (DIM >= 2) return launch25<DIM, VAR>(g, x, y, c1, c2, c3, ax, ay, az, s);
  const int nbx = (g.m1 + TX - 1) / TX;
  const int nby = (g.m2 + TY - 1) / TY;
  const int nbt = (g.n + TCHUNK - 1) / TCHUNK;
  const int64_t nblk = (int64_t)nbx * nby * g.m3 * nbt;
  if (nblk <= 0 || nblk > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_apply_L<DIM, VAR>), dim3((unsigned)nblk), dim3(TX, TY), 0, s, x, y, g.n,
                     g.m1, g.m2, g.m3, nbx, nby, nbt, c1, c2, c3, ax, ay, az);
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
