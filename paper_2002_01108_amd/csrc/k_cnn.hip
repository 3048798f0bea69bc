// Learned correction of the per-frequency inner solve: a 3-layer 3x3
// convolutional network, feature-wise modulated by lambda_k, that maps the
// residual left by one multigrid V-cycle to a correction (the V-cycle is the
// paper's inner solve, Section 4 and Section 5, Example 2; the network is an
// addition of this library).  Forward, backward and Adam kernels, FP32.
//
// Activations are [B][C][H][W] (one image per frequency block).  One thread
// per pixel computes every output channel of that pixel; the layer's weights
// sit in LDS and are read as broadcasts.  Weight gradients are summed over
// 16 x 16 pixel tiles staged in LDS (one partial per tile), then reduced in a
// fixed order, so training is deterministic.
#include "common.h"

namespace aao {
namespace {

constexpr int PT = 256;   // pixels per block for pixel-parallel kernels
constexpr int TILE = 16;  // weight-gradient tile edge

__device__ __forceinline__ float block_sum(float v, float* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  float s = 0.f;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;  // valid in thread 0
}

// MODE 0: hidden layer, z = conv(x), out = relu(gam * z + bet) (z stored if non-null)
// MODE 1: output layer, out = conv(x) + bias
template <int CI, int CO, int MODE>
__global__ __launch_bounds__(PT) void k_conv_fwd(const float* __restrict__ x,
                                                 const float* __restrict__ w,
                                                 const float* __restrict__ gam,
                                                 const float* __restrict__ bet,
                                                 const float* __restrict__ bias,
                                                 float* __restrict__ z, float* __restrict__ out,
                                                 int H, int W, int nchunk) {
  // weights staged tap-major, [c][di][dj][o], so that the CO weights of one
  // tap are contiguous (vector LDS reads, broadcast to the wave)
  __shared__ __align__(16) float ws[CI * 9 * CO];
  for (int t = threadIdx.x; t < CO * CI * 9; t += PT) {
    const int o = t / (CI * 9), tap = t - o * (CI * 9);
    ws[tap * CO + o] = w[t];
  }
  __syncthreads();
  const int HW = H * W;
  const int b = blockIdx.x / nchunk, chunk = blockIdx.x - b * nchunk;
  const int p = chunk * PT + threadIdx.x;
  if (p >= HW) return;
  const int i = p / W, j = p - i * W;
  // the 9 inputs of the next channel are loaded (from clamped in-range
  // addresses) while the current channel's taps are accumulated, and the taps
  // outside the image are zeroed afterwards, so loads overlap the arithmetic
  // instead of waiting one tap at a time behind a bounds test
  const int jm = j > 0 ? j - 1 : j, jp = j < W - 1 ? j + 1 : j;
  int rowoff[3];
  bool rok[3];
#pragma unroll
  for (int di = 0; di < 3; ++di) {
    const int ii = i + di - 1;
    rok[di] = ii >= 0 && ii < H;
    rowoff[di] = (rok[di] ? ii : i) * W;
  }
  bool tap_ok[9];
#pragma unroll
  for (int di = 0; di < 3; ++di) {
    tap_ok[3 * di] = rok[di] && j > 0;
    tap_ok[3 * di + 1] = rok[di];
    tap_ok[3 * di + 2] = rok[di] && j < W - 1;
  }
  auto load9 = [&](int c, float (&v)[9]) {
    const float* xc = x + ((int64_t)b * CI + c) * HW;
#pragma unroll
    for (int di = 0; di < 3; ++di) {
      v[3 * di] = xc[rowoff[di] + jm];
      v[3 * di + 1] = xc[rowoff[di] + j];
      v[3 * di + 2] = xc[rowoff[di] + jp];
    }
  };
  float acc[CO];
#pragma unroll
  for (int o = 0; o < CO; ++o) acc[o] = 0.f;
  float cur[9], nxt[9];
  load9(0, cur);
#pragma unroll 1
  for (int c = 0; c < CI; ++c) {
    if (c + 1 < CI) load9(c + 1, nxt);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const float vv = tap_ok[t] ? cur[t] : 0.f;
      const float* wt = ws + (c * 9 + t) * CO;
#pragma unroll
      for (int o = 0; o < CO; ++o) acc[o] += wt[o] * vv;
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) cur[t] = nxt[t];
  }
#pragma unroll
  for (int o = 0; o < CO; ++o) {
    const int64_t q = ((int64_t)b * CO + o) * HW + p;
    if (MODE == 0) {
      if (z) z[q] = acc[o];
      const float a = gam[b * CO + o] * acc[o] + bet[b * CO + o];
      out[q] = a > 0.f ? a : 0.f;
    } else {
      out[q] = acc[o] + bias[o];
    }
  }
}

// dx = adjoint of the convolution applied to dz
template <int CI, int CO>
__global__ __launch_bounds__(PT) void k_conv_bwd_data(const float* __restrict__ dz,
                                                      const float* __restrict__ w,
                                                      float* __restrict__ dx, int H, int W,
                                                      int nchunk) {
  __shared__ float ws[CO * CI * 9];
  for (int i = threadIdx.x; i < CO * CI * 9; i += PT) ws[i] = w[i];
  __syncthreads();
  const int HW = H * W;
  const int b = blockIdx.x / nchunk, chunk = blockIdx.x - b * nchunk;
  const int p = chunk * PT + threadIdx.x;
  if (p >= HW) return;
  const int i = p / W, j = p - i * W;
  float acc[CI];
#pragma unroll
  for (int c = 0; c < CI; ++c) acc[c] = 0.f;
#pragma unroll
  for (int o = 0; o < CO; ++o) {
    const float* g = dz + ((int64_t)b * CO + o) * HW;
#pragma unroll
    for (int di = 0; di < 3; ++di) {
      const int ii = i - di + 1;
      if (ii < 0 || ii >= H) continue;
#pragma unroll
      for (int dj = 0; dj < 3; ++dj) {
        const int jj = j - dj + 1;
        if (jj < 0 || jj >= W) continue;
        const float v = g[ii * W + jj];
#pragma unroll
        for (int c = 0; c < CI; ++c) acc[c] += ws[((o * CI + c) * 3 + di) * 3 + dj] * v;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CI; ++c) dx[((int64_t)b * CI + c) * HW + p] = acc[c];
}

// part[e * nparts + tile] = sum over the tile's pixels of dz[o] * x[c] shifted by the tap
template <int CI, int CO>
__global__ __launch_bounds__(PT) void k_conv_wgrad(const float* __restrict__ dz,
                                                   const float* __restrict__ x,
                                                   float* __restrict__ part, int H, int W,
                                                   int tx, int ty, int nparts) {
  __shared__ float sdz[CO][TILE * TILE];
  __shared__ float sx[CI][(TILE + 2) * (TILE + 2)];
  const int HW = H * W;
  const int per_b = tx * ty;
  const int b = blockIdx.x / per_b, t = blockIdx.x - b * per_b;
  const int i0 = (t / tx) * TILE, j0 = (t % tx) * TILE;
  for (int e = threadIdx.x; e < CO * TILE * TILE; e += PT) {
    const int o = e / (TILE * TILE), q = e - o * TILE * TILE;
    const int ii = i0 + q / TILE, jj = j0 + q % TILE;
    sdz[o][q] = (ii < H && jj < W) ? dz[((int64_t)b * CO + o) * HW + ii * W + jj] : 0.f;
  }
  for (int e = threadIdx.x; e < CI * (TILE + 2) * (TILE + 2); e += PT) {
    const int c = e / ((TILE + 2) * (TILE + 2)), q = e - c * (TILE + 2) * (TILE + 2);
    const int ii = i0 + q / (TILE + 2) - 1, jj = j0 + q % (TILE + 2) - 1;
    sx[c][q] = (ii >= 0 && ii < H && jj >= 0 && jj < W) ? x[((int64_t)b * CI + c) * HW + ii * W + jj]
                                                         : 0.f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < CO * CI * 9; e += PT) {
    const int o = e / (CI * 9), rem = e - o * CI * 9;
    const int c = rem / 9, tap = rem - c * 9, di = tap / 3, dj = tap - di * 3;
    float s = 0.f;
    for (int py = 0; py < TILE; ++py)
#pragma unroll 4
      for (int px = 0; px < TILE; ++px)
        s += sdz[o][py * TILE + px] * sx[c][(py + di) * (TILE + 2) + px + dj];
    part[(int64_t)e * nparts + blockIdx.x] = s;
  }
}

// FiLM + ReLU backward of a hidden layer: da = dh * (h > 0), dz = gam * da, and per
// (b, channel) partial sums of da*z (-> d gamma) and da (-> d beta).
template <int C>
__global__ __launch_bounds__(PT) void k_film_bwd(const float* __restrict__ dh,
                                                 const float* __restrict__ z,
                                                 const float* __restrict__ h,
                                                 const float* __restrict__ gam,
                                                 float* __restrict__ dz, float* __restrict__ part,
                                                 int HW, int nchunk) {
  __shared__ float red[PT / 64];
  const int b = blockIdx.x / nchunk, chunk = blockIdx.x - b * nchunk;
  const int p = chunk * PT + threadIdx.x;
  const bool ok = p < HW;
  for (int c = 0; c < C; ++c) {
    float sg = 0.f, sb = 0.f;
    if (ok) {
      const int64_t q = ((int64_t)b * C + c) * HW + p;
      const float da = h[q] > 0.f ? dh[q] : 0.f;
      dz[q] = gam[b * C + c] * da;
      sg = da * z[q];
      sb = da;
    }
    const float tg = block_sum(sg, red);
    const float tb = block_sum(sb, red);
    if (threadIdx.x == 0) {
      part[((int64_t)b * 2 * C + c) * nchunk + chunk] = tg;
      part[((int64_t)b * 2 * C + C + c) * nchunk + chunk] = tb;
    }
  }
}

// part[(c) * (B*nchunk) + b*nchunk + chunk] = partial sum of g[b][c] over the chunk
template <int C>
__global__ __launch_bounds__(PT) void k_chan_sum(const float* __restrict__ g,
                                                 float* __restrict__ part, int HW, int nchunk,
                                                 int nparts) {
  __shared__ float red[PT / 64];
  const int b = blockIdx.x / nchunk, chunk = blockIdx.x - b * nchunk;
  const int p = chunk * PT + threadIdx.x;
  for (int c = 0; c < C; ++c) {
    const float v = p < HW ? g[((int64_t)b * C + c) * HW + p] : 0.f;
    const float t = block_sum(v, red);
    if (threadIdx.x == 0) part[(int64_t)c * nparts + blockIdx.x] = t;
  }
}

// out[s] = sum_k part[s * n + k] (fixed order), optional scale; one block per segment
__global__ __launch_bounds__(PT) void k_seg_sum(const float* __restrict__ part, int n,
                                                float* __restrict__ out, float scale) {
  __shared__ float red[PT / 64];
  float s = 0.f;
  for (int k = threadIdx.x; k < n; k += PT) s += part[(int64_t)blockIdx.x * n + k];
  const float t = block_sum(s, red);
  if (threadIdx.x == 0) out[blockIdx.x] = t * scale;
}

// gamma = 1 + G phi, beta = H phi for both hidden layers; gb layout [4][B][C]
__global__ void k_film_params(const float* __restrict__ prm, const float* __restrict__ phi,
                              float* __restrict__ gb, int B, int C, int oG1, int oH1, int oG2,
                              int oH2) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 4 * B * C) return;
  const int which = idx / (B * C), r = idx - which * B * C, b = r / C, c = r - b * C;
  const int off = which == 0 ? oG1 : which == 1 ? oH1 : which == 2 ? oG2 : oH2;
  float s = 0.f;
  for (int f = 0; f < 4; ++f) s += prm[off + c * 4 + f] * phi[b * 4 + f];
  gb[idx] = (which == 0 || which == 2) ? 1.f + s : s;
}

// network features of each image's lambda_k: (Re, Im, log|lambda|, 1)
__global__ void k_cnn_features(const double* __restrict__ lam, float* __restrict__ phi, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const double re = lam[2 * b], im = lam[2 * b + 1];
  phi[4 * b] = (float)re;
  phi[4 * b + 1] = (float)im;
  phi[4 * b + 2] = (float)log(hypot(re, im));
  phi[4 * b + 3] = 1.f;
}

// dG[c][f] = sum_b dgam[b][c] phi[b][f]; dfilm layout [B][2C] (gam sums then beta sums)
__global__ void k_film_grad(const float* __restrict__ dfilm, const float* __restrict__ phi,
                            float* __restrict__ grad, int B, int C, int oG, int oH) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * C * 4) return;
  const int which = idx / (C * 4), r = idx - which * C * 4, c = r / 4, f = r - c * 4;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += dfilm[b * 2 * C + which * C + c] * phi[b * 4 + f];
  grad[(which == 0 ? oG : oH) + c * 4 + f] = s;
}

// ---------------------------------------------------------------- residual loss
// The correction y is followed by one red-black Gauss-Seidel sweep S for
// B e = rho (B = lambda_b I + tau K_a, face weights w = tau/h^2 a) and scored by
// ||rho - B S(y)||^2 / ||rho||^2.  Complex fields are [b][2][H][W] (Re, Im);
// lambda_b = (phi[4b], phi[4b+1]).  Red points: (i + j) even.
struct RsView {
  const float* wx;  // [H][W+1]
  const float* wy;  // [H+1][W]
  const float* phi;
  int H, W;
};

__device__ __forceinline__ void rs_nbr(const RsView& v, const float* re, const float* im, int i,
                                       int j, float& sr, float& si, float& d) {
  const int W = v.W, H = v.H;
  const float wl = v.wx[j * (W + 1) + i], wr = v.wx[j * (W + 1) + i + 1];
  const float wd = v.wy[j * W + i], wu = v.wy[(j + 1) * W + i];
  d = wl + wr + wd + wu;
  sr = si = 0.f;
  const int p = j * W + i;
  if (i > 0) { sr += wl * re[p - 1]; si += wl * im[p - 1]; }
  if (i < W - 1) { sr += wr * re[p + 1]; si += wr * im[p + 1]; }
  if (j > 0) { sr += wd * re[p - W]; si += wd * im[p - W]; }
  if (j < H - 1) { sr += wu * re[p + W]; si += wu * im[p + W]; }
}

// stage 0: e = y with the red points replaced by (rho + W y)/den    (red half sweep)
// stage 1: black points of e <- (rho + W e)/den                     (black half sweep)
// stage 2: q = rho - B e, partial sums of q^2, dq = 2 q / (rn_b B) into q
// stage 3: g = -B^H dq                                              (into out)
// stage 4: h = g + W (g / conj(den)) on red points, 0 on black      (adjoint of stage 1)
// stage 5: dy = W (h / conj(den)) on black points, 0 on red         (adjoint of stage 0)
// stage 6: out = in / (lambda + d)      (the network output scaled by the diagonal)
// stage 7: out = in / conj(lambda + d)  (adjoint of stage 6)
// (`in` and `out` alias in stages 1 and 7, so neither is restrict-qualified.)
__global__ __launch_bounds__(PT) void k_resid(RsView v, int stage, const float* in,
                                              const float* __restrict__ rho, float* out,
                                              const float* __restrict__ rn, float invB,
                                              float* __restrict__ part, int nchunk) {
  __shared__ float red[PT / 64];
  const int HW = v.H * v.W;
  const int b = blockIdx.x / nchunk, chunk = blockIdx.x - b * nchunk;
  const int p = chunk * PT + threadIdx.x;
  float acc = 0.f;
  if (p < HW) {
    const int j = p / v.W, i = p - j * v.W;
    const bool is_red = ((i + j) & 1) == 0;
    const float lr = v.phi[4 * b], li = v.phi[4 * b + 1];
    const int64_t o = (int64_t)b * 2 * HW;
    const float* ir = in + o;
    const float* ii = ir + HW;
    float* orr = out + o;
    float* oi = orr + HW;
    float sr, si, d;
    rs_nbr(v, ir, ii, i, j, sr, si, d);
    const float c = lr + d;
    const float inv = 1.f / (c * c + li * li);
    if (stage == 0 || stage == 1) {
      const bool upd = (stage == 0) ? is_red : !is_red;
      if (upd) {
        const float ar = rho[o + p] + sr, ai = rho[o + HW + p] + si;
        orr[p] = (ar * c + ai * li) * inv;
        oi[p] = (ai * c - ar * li) * inv;
      } else if (stage == 0) {
        orr[p] = ir[p];
        oi[p] = ii[p];
      }
    } else if (stage == 2) {
      const float er = ir[p], ei = ii[p];
      const float qr = rho[o + p] - (c * er - li * ei - sr);
      const float qi = rho[o + HW + p] - (c * ei + li * er - si);
      acc = qr * qr + qi * qi;
      const float sc = 2.f * invB / rn[b];
      orr[p] = sc * qr;
      oi[p] = sc * qi;
    } else if (stage == 3) {
      // B^H g = (conj(lambda) + D) g - W g
      const float gr = ir[p], gi = ii[p];
      orr[p] = -((c * gr + li * gi) - sr);
      oi[p] = -((c * gi - li * gr) - si);
    } else if (stage == 6) {
      const float yr = ir[p], yi = ii[p];
      orr[p] = (yr * c + yi * li) * inv;
      oi[p] = (yi * c - yr * li) * inv;
    } else if (stage == 7) {
      const float gr = ir[p], gi = ii[p];
      orr[p] = (gr * c - gi * li) * inv;
      oi[p] = (gi * c + gr * li) * inv;
    }
  }
  if (stage == 2) {
    const float t = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
  }
}

// stages 4 and 5: neighbour sums of x / conj(den) restricted to one colour
__global__ __launch_bounds__(PT) void k_resid_adj(RsView v, int stage, const float* __restrict__ g,
                                                  float* __restrict__ out, int nchunk) {
  const int HW = v.H * v.W, W = v.W, H = v.H;
  const int b = blockIdx.x / nchunk, chunk = blockIdx.x - b * nchunk;
  const int p = chunk * PT + threadIdx.x;
  if (p >= HW) return;
  const int j = p / W, i = p - j * W;
  const bool is_red = ((i + j) & 1) == 0;
  const float lr = v.phi[4 * b], li = v.phi[4 * b + 1];
  const int64_t o = (int64_t)b * 2 * HW;
  const float* gr = g + o;
  const float* gi = gr + HW;
  // x / conj(lambda + D_q) at neighbour q
  auto scaled = [&](int q, int qi_, int qj_, float& xr, float& xi) {
    const float dq = v.wx[qj_ * (W + 1) + qi_] + v.wx[qj_ * (W + 1) + qi_ + 1] +
                     v.wy[qj_ * W + qi_] + v.wy[(qj_ + 1) * W + qi_];
    const float c = lr + dq;
    const float inv = 1.f / (c * c + li * li);
    // (a + ib) / (c - i li) = (a + ib)(c + i li) / |.|^2
    xr = (gr[q] * c - gi[q] * li) * inv;
    xi = (gi[q] * c + gr[q] * li) * inv;
  };
  const bool active = (stage == 4) ? is_red : !is_red;
  float sr = 0.f, si = 0.f;
  if (active) {
    const float wl = v.wx[j * (W + 1) + i], wr = v.wx[j * (W + 1) + i + 1];
    const float wd = v.wy[j * W + i], wu = v.wy[(j + 1) * W + i];
    float xr, xi;
    if (i > 0) { scaled(p - 1, i - 1, j, xr, xi); sr += wl * xr; si += wl * xi; }
    if (i < W - 1) { scaled(p + 1, i + 1, j, xr, xi); sr += wr * xr; si += wr * xi; }
    if (j > 0) { scaled(p - W, i, j - 1, xr, xi); sr += wd * xr; si += wd * xi; }
    if (j < H - 1) { scaled(p + W, i, j + 1, xr, xi); sr += wu * xr; si += wu * xi; }
    if (stage == 4) { sr += gr[p]; si += gi[p]; }
  }
  out[o + p] = sr;
  out[o + HW + p] = si;
}

__global__ void k_loss_final(const float* __restrict__ lb, const float* __restrict__ tn, int B,
                             float* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += lb[b] / tn[b];
    *out = s / (float)B;
  }
}

__global__ void k_adam(float* __restrict__ prm, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int np, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  prm[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// gather a training batch from the stored pairs: network input X = (rho, log a)
// and R = rho alone (the right-hand side of the residual loss)
__global__ void k_gather(const float* __restrict__ px, const float* __restrict__ pphi,
                         const float* __restrict__ ptn, const float* __restrict__ loga,
                         const int* __restrict__ idx, float* __restrict__ X,
                         float* __restrict__ R, float* __restrict__ phi, float* __restrict__ tn,
                         int B, int HW) {
  const int64_t total = (int64_t)B * HW;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / HW);
    const int p = (int)(e - (int64_t)b * HW);
    const int64_t src = (int64_t)idx[b] * 2 * HW;
    const float r0 = px[src + p], r1 = px[src + HW + p];
    X[((int64_t)b * 3 + 0) * HW + p] = r0;
    X[((int64_t)b * 3 + 1) * HW + p] = r1;
    X[((int64_t)b * 3 + 2) * HW + p] = loga[p];
    R[((int64_t)b * 2 + 0) * HW + p] = r0;
    R[((int64_t)b * 2 + 1) * HW + p] = r1;
    if (p == 0) {
      for (int f = 0; f < 4; ++f) phi[b * 4 + f] = pphi[idx[b] * 4 + f];
      tn[b] = ptn[idx[b]];
    }
  }
}

// ---------------------------------------------------------------- spectrum <-> images
// per block sum of squares over both planes of the m x m valid region
template <typename T>
__global__ __launch_bounds__(PT) void k_block_sumsq(MgGrid v, int m, float* __restrict__ part,
                                                    int nchunk) {
  __shared__ float red[PT / 64];
  const int k = blockIdx.x / nchunk, chunk = blockIdx.x - k * nchunk;
  const int p = chunk * PT + threadIdx.x;
  float s = 0.f;
  if (p < m * m) {
    const int j = p / m, i = p - j * m;
    const T* q = (const T*)v.p + k * v.bstride + (int64_t)j * v.pitch + i;
    const float a = (float)q[0], b = (float)q[v.pstride];
    s = a * a + b * b;
  }
  const float t = block_sum(s, red);
  if (threadIdx.x == 0) part[(int64_t)k * nchunk + chunk] = t;
}

// X[k] = (Re rho / s_k, Im rho / s_k, loga), s_k = sqrt(ss_k / (2 m^2)); zeros if s_k = 0
template <typename T>
__global__ void k_pack_input(MgGrid v, const float* __restrict__ ss,
                             const float* __restrict__ loga, float* __restrict__ X, int m,
                             int nh, int nch) {
  const int64_t HW = (int64_t)m * m, total = (int64_t)nh * HW;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(e / HW);
    const int p = (int)(e - (int64_t)k * HW);
    const int j = p / m, i = p - j * m;
    const float s = sqrtf(ss[k] / (2.f * (float)HW));
    const float inv = s > 0.f ? 1.f / s : 0.f;
    const T* q = (const T*)v.p + k * v.bstride + (int64_t)j * v.pitch + i;
    X[((int64_t)k * nch + 0) * HW + p] = (float)q[0] * inv;
    X[((int64_t)k * nch + 1) * HW + p] = (float)q[v.pstride] * inv;
    if (nch == 3) X[((int64_t)k * nch + 2) * HW + p] = loga[p];
  }
}

// e[k] += s_k * Y[k] / (lambda_k + d) on the valid region, d the diagonal of
// tau K_a (sum of the four face weights wx [m][m+1], wy [m+1][m])
template <typename T>
__global__ void k_unpack_add(const float* __restrict__ Y, const float* __restrict__ ss, MgGrid v,
                             MgGrid vo, const double* __restrict__ lam,
                             const float* __restrict__ wx, const float* __restrict__ wy, int m,
                             int nh) {
  const int64_t HW = (int64_t)m * m, total = (int64_t)nh * HW;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(e / HW);
    const int p = (int)(e - (int64_t)k * HW);
    const int j = p / m, i = p - j * m;
    const float s = sqrtf(ss[k] / (2.f * (float)HW));
    const float d = wx[j * (m + 1) + i] + wx[j * (m + 1) + i + 1] + wy[j * m + i] + wy[(j + 1) * m + i];
    const float c = (float)lam[2 * k] + d, li = (float)lam[2 * k + 1];
    const float inv = s / (c * c + li * li);
    const float yr = Y[((int64_t)k * 2 + 0) * HW + p], yi = Y[((int64_t)k * 2 + 1) * HW + p];
    const T* q = (const T*)v.p + k * v.bstride + (int64_t)j * v.pitch + i;
    T* qo = (T*)vo.p + k * vo.bstride + (int64_t)j * vo.pitch + i;
    qo[0] = q[0] + (T)((yr * c + yi * li) * inv);
    qo[vo.pstride] = q[v.pstride] + (T)((yi * c - yr * li) * inv);
  }
}

unsigned grid1(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

// ---------------------------------------------------------------- launchers
int cnn_chunks(int HW) { return (HW + PT - 1) / PT; }
int cnn_tiles(int H, int W) { return ((H + TILE - 1) / TILE) * ((W + TILE - 1) / TILE); }

hipError_t cnn_conv_fwd(int layer, const float* x, const float* w, const float* gam,
                        const float* bet, const float* bias, float* z, float* out, int B, int H,
                        int W, hipStream_t s) {
  const int nchunk = cnn_chunks(H * W);
  const dim3 grid((unsigned)(B * nchunk));
  if (layer == 1)
    hipLaunchKernelGGL((k_conv_fwd<3, kCnnC, 0>), grid, dim3(PT), 0, s, x, w, gam, bet, bias, z,
                       out, H, W, nchunk);
  else if (layer == 2)
    hipLaunchKernelGGL((k_conv_fwd<kCnnC, kCnnC, 0>), grid, dim3(PT), 0, s, x, w, gam, bet, bias,
                       z, out, H, W, nchunk);
  else
    hipLaunchKernelGGL((k_conv_fwd<kCnnC, 2, 1>), grid, dim3(PT), 0, s, x, w, gam, bet, bias, z,
                       out, H, W, nchunk);
  return hipGetLastError();
}

hipError_t cnn_conv_bwd_data(int layer, const float* dz, const float* w, float* dx, int B, int H,
                             int W, hipStream_t s) {
  const int nchunk = cnn_chunks(H * W);
  const dim3 grid((unsigned)(B * nchunk));
  if (layer == 1)
    hipLaunchKernelGGL((k_conv_bwd_data<3, kCnnC>), grid, dim3(PT), 0, s, dz, w, dx, H, W, nchunk);
  else if (layer == 2)
    hipLaunchKernelGGL((k_conv_bwd_data<kCnnC, kCnnC>), grid, dim3(PT), 0, s, dz, w, dx, H, W,
                       nchunk);
  else
    hipLaunchKernelGGL((k_conv_bwd_data<kCnnC, 2>), grid, dim3(PT), 0, s, dz, w, dx, H, W, nchunk);
  return hipGetLastError();
}

// weight gradient of layer `layer` into grad (length CO*CI*9), via partials in `part`
hipError_t cnn_conv_wgrad(int layer, const float* dz, const float* x, float* part, float* grad,
                          int B, int H, int W, hipStream_t s) {
  const int tx = (W + TILE - 1) / TILE, ty = (H + TILE - 1) / TILE;
  const int nparts = B * tx * ty;
  int nw;
  if (layer == 1) {
    nw = kCnnC * 3 * 9;
    hipLaunchKernelGGL((k_conv_wgrad<3, kCnnC>), dim3(nparts), dim3(PT), 0, s, dz, x, part, H, W,
                       tx, ty, nparts);
  } else if (layer == 2) {
    nw = kCnnC * kCnnC * 9;
    hipLaunchKernelGGL((k_conv_wgrad<kCnnC, kCnnC>), dim3(nparts), dim3(PT), 0, s, dz, x, part, H,
                       W, tx, ty, nparts);
  } else {
    nw = 2 * kCnnC * 9;
    hipLaunchKernelGGL((k_conv_wgrad<kCnnC, 2>), dim3(nparts), dim3(PT), 0, s, dz, x, part, H, W,
                       tx, ty, nparts);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_seg_sum, dim3(nw), dim3(PT), 0, s, part, nparts, grad, 1.0f);
  return hipGetLastError();
}

// FiLM/ReLU backward of hidden layer; dfilm receives [B][2C] (d gamma, d beta)
hipError_t cnn_film_bwd(const float* dh, const float* z, const float* h, const float* gam,
                        float* dz, float* part, float* dfilm, int B, int H, int W,
                        hipStream_t s) {
  const int nchunk = cnn_chunks(H * W);
  hipLaunchKernelGGL((k_film_bwd<kCnnC>), dim3((unsigned)(B * nchunk)), dim3(PT), 0, s, dh, z, h,
                     gam, dz, part, H * W, nchunk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_seg_sum, dim3((unsigned)(B * 2 * kCnnC)), dim3(PT), 0, s, part, nchunk,
                     dfilm, 1.0f);
  return hipGetLastError();
}

hipError_t cnn_bias_grad(const float* dy, float* part, float* grad, int B, int H, int W,
                         hipStream_t s) {
  const int nchunk = cnn_chunks(H * W);
  const int nparts = B * nchunk;
  hipLaunchKernelGGL((k_chan_sum<2>), dim3((unsigned)nparts), dim3(PT), 0, s, dy, part, H * W,
                     nchunk, nparts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_seg_sum, dim3(2), dim3(PT), 0, s, part, nparts, grad, 1.0f);
  return hipGetLastError();
}

hipError_t cnn_film_params(const float* prm, const float* phi, float* gb, int B, hipStream_t s) {
  const int total = 4 * B * kCnnC;
  hipLaunchKernelGGL(k_film_params, dim3((total + 255) / 256), dim3(256), 0, s, prm, phi, gb, B,
                     kCnnC, kCnnOffG1, kCnnOffH1, kCnnOffG2, kCnnOffH2);
  return hipGetLastError();
}

hipError_t cnn_features(const double* lam, float* phi, int B, hipStream_t s) {
  hipLaunchKernelGGL(k_cnn_features, dim3((B + 255) / 256), dim3(256), 0, s, lam, phi, B);
  return hipGetLastError();
}

hipError_t cnn_film_grad(const float* dfilm, const float* phi, float* grad, int B, int layer,
                         hipStream_t s) {
  const int oG = layer == 1 ? kCnnOffG1 : kCnnOffG2, oH = layer == 1 ? kCnnOffH1 : kCnnOffH2;
  hipLaunchKernelGGL(k_film_grad, dim3(1), dim3(256), 0, s, dfilm, phi, grad, B, kCnnC, oG, oH);
  return hipGetLastError();
}

// Residual loss of the correction y for B e = rho after one red-black sweep;
// loss value into *out, gradient in y into dy.  E, Q, G, Hb: [B][2][H][W] scratch.
hipError_t cnn_resid_loss(const float* y, const float* rho, const float* rn, const float* phi,
                          const float* wx, const float* wy, float* E, float* Q, float* G,
                          float* Hb, float* dy, float* part, float* lb, float* out, int B, int H,
                          int W, hipStream_t s) {
  const int nchunk = cnn_chunks(H * W);
  const dim3 grid((unsigned)(B * nchunk)), blk(PT);
  const RsView v{wx, wy, phi, H, W};
  const float invB = 1.0f / (float)B;
  hipLaunchKernelGGL(k_resid, grid, blk, 0, s, v, 6, y, rho, G, rn, invB, part, nchunk);
  hipLaunchKernelGGL(k_resid, grid, blk, 0, s, v, 0, G, rho, E, rn, invB, part, nchunk);
  hipLaunchKernelGGL(k_resid, grid, blk, 0, s, v, 1, E, rho, E, rn, invB, part, nchunk);
  hipLaunchKernelGGL(k_resid, grid, blk, 0, s, v, 2, E, rho, Q, rn, invB, part, nchunk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_seg_sum, dim3((unsigned)B), blk, 0, s, part, nchunk, lb, 1.0f);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, lb, rn, B, out);
  hipLaunchKernelGGL(k_resid, grid, blk, 0, s, v, 3, Q, rho, G, rn, invB, part, nchunk);
  hipLaunchKernelGGL(k_resid_adj, grid, blk, 0, s, v, 4, G, Hb, nchunk);
  hipLaunchKernelGGL(k_resid_adj, grid, blk, 0, s, v, 5, Hb, dy, nchunk);
  hipLaunchKernelGGL(k_resid, grid, blk, 0, s, v, 7, dy, rho, dy, rn, invB, part, nchunk);
  return hipGetLastError();
}

hipError_t cnn_adam(float* prm, const float* g, float* m, float* v, int np, float lr, int step,
                    hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((np + 255) / 256), dim3(256), 0, s, prm, g, m, v, np, lr, b1, b2,
                     eps, c1, c2);
  return hipGetLastError();
}

hipError_t cnn_gather(const float* px, const float* pphi, const float* ptn, const float* loga,
                      const int* idx, float* X, float* R, float* phi, float* tn, int B, int HW,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3(grid1((int64_t)B * HW)), dim3(256), 0, s, px, pphi, ptn, loga,
                     idx, X, R, phi, tn, B, HW);
  return hipGetLastError();
}

template <typename T>
hipError_t cnn_block_sumsq(const MgGrid& v, int m, int nh, float* part, float* out,
                           hipStream_t s) {
  const int nchunk = cnn_chunks(m * m);
  hipLaunchKernelGGL((k_block_sumsq<T>), dim3((unsigned)(nh * nchunk)), dim3(PT), 0, s, v, m,
                     part, nchunk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_seg_sum, dim3((unsigned)nh), dim3(PT), 0, s, part, nchunk, out, 1.0f);
  return hipGetLastError();
}

template <typename T>
hipError_t cnn_pack_input(const MgGrid& v, const float* ss, const float* loga, float* X, int m,
                          int nh, int nch, hipStream_t s) {
  hipLaunchKernelGGL((k_pack_input<T>), dim3(grid1((int64_t)nh * m * m)), dim3(256), 0, s, v, ss,
                     loga, X, m, nh, nch);
  return hipGetLastError();
}

template <typename T>
hipError_t cnn_unpack_add(const float* Y, const float* ss, const MgGrid& v, const MgGrid& vo,
                          const double* lam, const float* wx, const float* wy, int m, int nh,
                          hipStream_t s) {
  hipLaunchKernelGGL((k_unpack_add<T>), dim3(grid1((int64_t)nh * m * m)), dim3(256), 0, s, Y, ss,
                     v, vo, lam, wx, wy, m, nh);
  return hipGetLastError();
}

#define INST(T)                                                                              \
  template hipError_t cnn_block_sumsq<T>(const MgGrid&, int, int, float*, float*, hipStream_t); \
  template hipError_t cnn_pack_input<T>(const MgGrid&, const float*, const float*, float*, int, \
                                        int, int, hipStream_t);                              \
  template hipError_t cnn_unpack_add<T>(const float*, const float*, const MgGrid&,             \
                                        const MgGrid&, const double*, const float*, const float*, \
                                        int, int, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace aao
