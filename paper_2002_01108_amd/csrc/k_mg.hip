// Geometric multigrid V-cycle on the shifted blocks B_k = lambda_k I + tau K_a
// of Step 2 (Section 4, eq. (blockdiaginv)) when the coefficient varies and
// the blocks no longer diagonalise by sine transforms; the paper applies one
// V-cycle with one pre- and one post-smoothing step, linear interpolation and
// its transpose (Section 4, closing paragraphs; Section 5, Example 2).
//
// All n/2+1 blocks are processed by every launch.  Smoother: red-black
// Gauss-Seidel (red: i1 + i2 even), one red and one black half sweep per
// launch (tiled, see k_rbgs_fused), which also restricts the residual after
// pre-smoothing and adds the prolonged coarse correction before
// post-smoothing; the stand-alone residual (learned correction) takes one
// thread per grid point and block.
// Restriction: full weighting (transpose of bilinear interpolation / 4).
// Prolongation: bilinear.  Coarse operators are rediscretised on the host:
// face weights w = tau/h_l^2 * a with harmonic face averages (flux form), or
// the four coupling planes tau (W, E, S, N) of a nonsymmetric five-point
// operator (wy == nullptr; upwinded convection-diffusion with the wind taken
// at the coarse nodes).
//
// A grid view addresses element (k, plane, j, i) at
//   p + k*bstride + plane*pstride + j*pitch + i
// so the finest level works in place on the padded split-plane spectrum.
#include "common.h"

namespace aao {
namespace {

template <typename T> struct GView {
  T* p;
  int pitch;
  int64_t pstride, bstride;
  __device__ __forceinline__ T* at(int k, int j, int i) const {
    return p + k * bstride + (int64_t)j * pitch + i;
  }
};

// bilinear interpolation of the coarse grid c at fine node (j, i): coarse node
// I sits on fine node 2I+1; zero beyond the coarse grid
template <typename T>
__device__ __forceinline__ void interp(const GView<T>& c, int k, int j, int i, int mc, T& ar,
                                       T& ai) {
  int Ix[2], Jy[2];
  T wxv[2], wyv[2];
  int nx, ny;
  if (i & 1) { Ix[0] = (i - 1) >> 1; wxv[0] = T(1); nx = 1; }
  else { Ix[0] = (i >> 1) - 1; Ix[1] = i >> 1; wxv[0] = wxv[1] = T(0.5); nx = 2; }
  if (j & 1) { Jy[0] = (j - 1) >> 1; wyv[0] = T(1); ny = 1; }
  else { Jy[0] = (j >> 1) - 1; Jy[1] = j >> 1; wyv[0] = wyv[1] = T(0.5); ny = 2; }
  ar = T(0);
  ai = T(0);
  for (int b = 0; b < ny; ++b) {
    if (Jy[b] < 0 || Jy[b] >= mc) continue;
    for (int a = 0; a < nx; ++a) {
      if (Ix[a] < 0 || Ix[a] >= mc) continue;
      const T w = wxv[a] * wyv[b];
      const T* cp = c.at(k, Jy[b], Ix[a]);
      ar += w * cp[0];
      ai += w * cp[c.pstride];
    }
  }
}

// couplings of node (j, i) to its west, east, south and north neighbours
template <typename T>
__device__ __forceinline__ void couplings(const T* __restrict__ wx, const T* __restrict__ wy,
                                          int j, int i, int m, T& wl, T& wr, T& wd, T& wu) {
  if (wy) {
    wl = wx[(int64_t)j * (m + 1) + i];
    wr = wx[(int64_t)j * (m + 1) + i + 1];
    wd = wy[(int64_t)j * m + i];
    wu = wy[(int64_t)(j + 1) * m + i];
  } else {
    const int64_t p = (int64_t)j * m + i, mm = (int64_t)m * m;
    wl = wx[p];
    wr = wx[p + mm];
    wd = wx[p + 2 * mm];
    wu = wx[p + 3 * mm];
  }
}

// sum of coupling * e_nbr (complex) and the diagonal (sum of couplings) at (j, i)
template <typename T>
__device__ __forceinline__ void nbr_sum(const GView<T>& e, int k, int j, int i, int m,
                                        const T* __restrict__ wx, const T* __restrict__ wy,
                                        T& sr, T& si, T& d) {
  T wl, wr, wd, wu;
  couplings(wx, wy, j, i, m, wl, wr, wd, wu);
  d = wl + wr + wd + wu;
  sr = T(0);
  si = T(0);
  const T* c = e.at(k, j, i);
  const int64_t ps = e.pstride;
  if (i > 0) { sr += wl * c[-1]; si += wl * c[ps - 1]; }
  if (i < m - 1) { sr += wr * c[1]; si += wr * c[ps + 1]; }
  if (j > 0) { sr += wd * c[-e.pitch]; si += wd * c[ps - e.pitch]; }
  if (j < m - 1) { sr += wu * c[e.pitch]; si += wu * c[ps + e.pitch]; }
}

// res = r - (lambda + d) e + s
template <typename T>
__global__ void k_residual(GView<T> e, GView<T> r, GView<T> res, const T* __restrict__ wx,
                           const T* __restrict__ wy, const double* __restrict__ lam, int m,
                           int nh) {
  const int64_t total = (int64_t)nh * m * m;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(idx / ((int64_t)m * m));
    const int rem = (int)(idx - (int64_t)k * m * m);
    const int j = rem / m, i = rem - j * m;
    T sr, si, d;
    nbr_sum(e, k, j, i, m, wx, wy, sr, si, d);
    const T* ep = e.at(k, j, i);
    const T* rp = r.at(k, j, i);
    const T c = (T)lam[2 * k] + d, dd = (T)lam[2 * k + 1];
    const T er = ep[0], ei = ep[e.pstride];
    T* op = res.at(k, j, i);
    op[0] = rp[0] - (c * er - dd * ei) + sr;
    op[res.pstride] = rp[r.pstride] - (c * ei + dd * er) + si;
  }
}

// One smoothing step (a red then a black half sweep) in one pass over the
// data.  A block owns a FTX x FTY tile of one frequency block: e (old values)
// and r are staged in LDS with halos, the red points are updated on the tile
// plus a ring of EH - 1, the black points on the tile plus EH - 2 (their red
// neighbours are then all new).  The halo rings repeat the neighbouring tiles'
// updates with the same inputs, so every point gets the value the two separate
// half sweeps give.  Outside the grid e and r are zero (Dirichlet).  The old
// iterate is read from e and the new one written to eo: blocks read their
// neighbours' old values, so eo may equal e only when the old iterate is zero
// (zero_init, e unread).  With mc > 0 the old iterate is e plus the bilinear
// interpolation of the coarse-grid correction ec (the prolongation of the
// V-cycle, added while the tile is staged).
// RST (pre-smoothing): the halos grow by one, the residual r - B e is formed on
// the tile plus one ring in LDS, and its full-weighting restriction is written
// for the coarse points centred in the tile (fine node 2J+1, 2I+1; the tile
// origin is even, so each coarse point has exactly one owner).
constexpr int FTX = 32, FTY = 16;   // tile shape measured fastest of 16..128 x 8..32
static_assert(FTX % 2 == 0 && FTY % 2 == 0, "even tile origins");

template <typename T, bool RST>
__global__ __launch_bounds__(256) void k_rbgs_fused(GView<T> e, GView<T> eo, GView<T> r,
                                                    GView<T> rc, int mcr, GView<T> ec, int mc,
                                                    const T* __restrict__ wx,
                                                    const T* __restrict__ wy,
                                                    const double* __restrict__ lam, int m,
                                                    int zero_init) {
  constexpr int EH = RST ? 4 : 3, EX = FTX + 2 * EH, EY = FTY + 2 * EH;   // e tile + halo
  constexpr int RH = EH - 1, RX = FTX + 2 * RH, RY = FTY + 2 * RH;        // r tile + halo
  constexpr int QX = RST ? FTX + 2 : 1, QY = RST ? FTY + 2 : 1;           // residual, ring 1
  __shared__ T se[2][EY][EX];
  __shared__ T sr[2][RY][RX];
  __shared__ T sq[2][QY][QX];
  const int k = blockIdx.z;
  const int x0 = blockIdx.x * FTX, y0 = blockIdx.y * FTY;
  const T lr = (T)lam[2 * k], li = (T)lam[2 * k + 1];
  for (int q = threadIdx.x; q < EY * EX; q += 256) {
    const int ly = q / EX, lx = q % EX;
    const int j = y0 - EH + ly, i = x0 - EH + lx;
    T vr = T(0), vi = T(0);
    if (!zero_init && j >= 0 && j < m && i >= 0 && i < m) {
      const T* p = e.at(k, j, i);
      vr = p[0];
      vi = p[e.pstride];
      if (mc > 0) {
        T pr, pi;
        interp(ec, k, j, i, mc, pr, pi);
        vr = vr + pr;
        vi = vi + pi;
      }
    }
    se[0][ly][lx] = vr;
    se[1][ly][lx] = vi;
  }
  for (int q = threadIdx.x; q < RY * RX; q += 256) {
    const int ly = q / RX, lx = q % RX;
    const int j = y0 - RH + ly, i = x0 - RH + lx;
    T vr = T(0), vi = T(0);
    if (j >= 0 && j < m && i >= 0 && i < m) {
      const T* p = r.at(k, j, i);
      vr = p[0];
      vi = p[r.pstride];
    }
    sr[0][ly][lx] = vr;
    sr[1][ly][lx] = vi;
  }
  __syncthreads();
  // sum of couplings x neighbours and the diagonal at e-tile position (ey, ex)
  auto nsum = [&](int j, int i, int ey, int ex, T& snr, T& sni, T& d) {
    T wl, wr, wd, wu;
    couplings(wx, wy, j, i, m, wl, wr, wd, wu);
    d = wl + wr + wd + wu;
    snr = wl * se[0][ey][ex - 1] + wr * se[0][ey][ex + 1] + wd * se[0][ey - 1][ex] +
          wu * se[0][ey + 1][ex];
    sni = wl * se[1][ey][ex - 1] + wr * se[1][ey][ex + 1] + wd * se[1][ey - 1][ex] +
          wu * se[1][ey + 1][ex];
  };
  // Gauss-Seidel update of the points of one colour in the tile plus a ring
  // of `ring`: e = (r + sum of couplings x neighbours) / (lambda + diagonal)
  auto half_sweep = [&](int color, int ring) {
    const int W = FTX + 2 * ring, H = FTY + 2 * ring;
    for (int q = threadIdx.x; q < W * H; q += 256) {
      const int qy = q / W, qx = q - qy * W;
      const int j = y0 - ring + qy, i = x0 - ring + qx;
      if (j < 0 || j >= m || i < 0 || i >= m || ((i + j) & 1) != color) continue;
      const int ey = qy - ring + EH, ex = qx - ring + EH;
      T snr, sni, d;
      nsum(j, i, ey, ex, snr, sni, d);
      const int ry = qy - ring + RH, rx = qx - ring + RH;
      const T ar = sr[0][ry][rx] + snr, ai = sr[1][ry][rx] + sni;
      const T c = lr + d, dd = li;
      const T inv = T(1) / (c * c + dd * dd);
      se[0][ey][ex] = (ar * c + ai * dd) * inv;
      se[1][ey][ex] = (ai * c - ar * dd) * inv;
    }
  };
  half_sweep(0, EH - 1);
  __syncthreads();
  half_sweep(1, EH - 2);
  __syncthreads();
  if (RST) {   // residual r - B e on the tile plus one ring (zero outside the grid)
    for (int q = threadIdx.x; q < QX * QY; q += 256) {
      const int qy = q / QX, qx = q % QX;
      const int j = y0 - 1 + qy, i = x0 - 1 + qx;
      T vr = T(0), vi = T(0);
      if (j >= 0 && j < m && i >= 0 && i < m) {
        const int ey = qy - 1 + EH, ex = qx - 1 + EH;
        T snr, sni, d;
        nsum(j, i, ey, ex, snr, sni, d);
        const T er = se[0][ey][ex], ei = se[1][ey][ex];
        const T c = lr + d, dd = li;
        vr = sr[0][qy - 1 + RH][qx - 1 + RH] - (c * er - dd * ei) + snr;
        vi = sr[1][qy - 1 + RH][qx - 1 + RH] - (c * ei + dd * er) + sni;
      }
      sq[0][qy][qx] = vr;
      sq[1][qy][qx] = vi;
    }
  }
  for (int q = threadIdx.x; q < FTX * FTY; q += 256) {
    const int qy = q / FTX, qx = q % FTX;
    const int j = y0 + qy, i = x0 + qx;
    if (j >= m || i >= m) continue;
    T* ep = eo.at(k, j, i);
    ep[0] = se[0][qy + EH][qx + EH];
    ep[eo.pstride] = se[1][qy + EH][qx + EH];
  }
  if (RST) {
    __syncthreads();
    // coarse (J, I) = (1/16) [4 centre + 2 (edge neighbours) + corners] of the
    // residual around fine node (2J+1, 2I+1)
    constexpr int CX = FTX / 2, CY = FTY / 2;
    for (int q = threadIdx.x; q < CX * CY; q += 256) {
      const int J = y0 / 2 + q / CX, I = x0 / 2 + q % CX;
      if (J >= mcr || I >= mcr) continue;
      const int ly = 2 * J + 1 - y0 + 1, lx = 2 * I + 1 - x0 + 1;
      for (int pl = 0; pl < 2; ++pl) {
        const T v = T(4) * sq[pl][ly][lx] +
                    T(2) * (sq[pl][ly][lx - 1] + sq[pl][ly][lx + 1] + sq[pl][ly - 1][lx] +
                            sq[pl][ly + 1][lx]) +
                    (sq[pl][ly - 1][lx - 1] + sq[pl][ly - 1][lx + 1] + sq[pl][ly + 1][lx - 1] +
                     sq[pl][ly + 1][lx + 1]);
        rc.at(k, J, I)[pl * rc.pstride] = v * T(0.0625);
      }
    }
  }
}

unsigned mg_grid(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

template <typename T> GView<T> view(const MgGrid& g) {
  return GView<T>{(T*)g.p, g.pitch, g.pstride, g.bstride};
}

}  // namespace

template <typename T>
hipError_t mg_sweep(const MgGrid& e, const MgGrid& eo, const MgGrid& r, const MgGrid* rc,
                    int mcr, const MgGrid* ec, int mc, const void* wx, const void* wy,
                    const double* lam, int m, int nh, int zero_init, hipStream_t s) {
  if (m < 1 || nh < 1 || nh > 65535) return hipErrorInvalidValue;
  if (!zero_init && e.p == eo.p) return hipErrorInvalidValue;   // blocks read old values
  if ((ec != nullptr) != (mc > 0) || (ec && 2 * mc + 1 > m)) return hipErrorInvalidValue;
  if ((rc != nullptr) != (mcr > 0) || (rc && 2 * mcr + 1 > m)) return hipErrorInvalidValue;
  const dim3 grid((m + FTX - 1) / FTX, (m + FTY - 1) / FTY, nh);
  const GView<T> vc = ec ? view<T>(*ec) : view<T>(e);
  if (rc)
    hipLaunchKernelGGL((k_rbgs_fused<T, true>), grid, dim3(256), 0, s, view<T>(e), view<T>(eo),
                       view<T>(r), view<T>(*rc), mcr, vc, ec ? mc : 0, (const T*)wx,
                       (const T*)wy, lam, m, zero_init);
  else
    hipLaunchKernelGGL((k_rbgs_fused<T, false>), grid, dim3(256), 0, s, view<T>(e),
                       view<T>(eo), view<T>(r), view<T>(eo), 0, vc, ec ? mc : 0, (const T*)wx,
                       (const T*)wy, lam, m, zero_init);
  return hipGetLastError();
}

template <typename T>
hipError_t mg_residual(const MgGrid& e, const MgGrid& r, const MgGrid& res, const void* wx,
                       const void* wy, const double* lam, int m, int nh, hipStream_t s) {
  hipLaunchKernelGGL((k_residual<T>), dim3(mg_grid((int64_t)nh * m * m)), dim3(256), 0, s,
                     view<T>(e), view<T>(r), view<T>(res), (const T*)wx, (const T*)wy, lam, m, nh);
  return hipGetLastError();
}

#define INST(T)                                                                                 \
  template hipError_t mg_sweep<T>(const MgGrid&, const MgGrid&, const MgGrid&, const MgGrid*, \
                                  int, const MgGrid*, int, const void*, const void*,           \
                                  const double*, int, int, int, hipStream_t);                  \
  template hipError_t mg_residual<T>(const MgGrid&, const MgGrid&, const MgGrid&, const void*, \
                                     const void*, const double*, int, int, hipStream_t);

INST(double)
INST(float)
#undef INST

}  // namespace aao
