// Internal declarations shared by the HIP kernels and the host side of the
// all-at-once BEC library.  Not part of the public C ABI (include/aao.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/aao.h"

namespace aao {

// ---------------------------------------------------------------- complex helpers
template <typename T> struct cplx { T x, y; };

template <typename T> __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename T> __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) {
  return {a.x - b.x, a.y - b.y};
}
template <typename T> __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// Hardware places workgroup b on XCD b % 8, and each XCD has its own L2.  This
// maps the hardware index to a logical tile index so that every XCD gets one
// contiguous run of logical tiles (neighbouring tiles share cache lines and
// operands in one L2).  A bijection for any nblk: the first nblk % 8 XCDs get
// one extra tile.
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
  const int q = nblk / 8, r = nblk % 8;
  const int xcd = bid % 8, slot = bid / 8;
  return xcd * q + (xcd < r ? xcd : r) + slot;
}

// Persistent grids: as many blocks as fit on the chip at once (a multiple of
// 8); block b runs on XCD b % 8 (round-robin dispatch), and XCD x walks a
// contiguous range of the n work items so that neighbouring items share its
// L2.  Work item loops are uniform per block (barriers inside are fine).
struct StripRange {
  int first, end, step;
};
__device__ __forceinline__ StripRange xcd_strips(int n) {
  const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8, per = gridDim.x / 8;
  const int q = n / 8, r = n % 8;
  const int lo = xcd * q + (xcd < r ? xcd : r);
  return {lo + slot, lo + q + (xcd < r ? 1 : 0), per};
}

// Blocks of one kernel resident on the whole chip at once, rounded down to a
// multiple of 8 (the walk above assumes it); -1 if the runtime cannot say.
template <typename K>
int persistent_grid(K kernel, int threads) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess)
    return -1;
  const int g = (cus * per_cu) / 8 * 8;
  return g >= 8 ? g : -1;
}

// grid for n work items: the resident count, or fewer when there are fewer items
inline int strip_grid(int resident, int64_t n) {
  const int64_t cover = (n + 7) / 8 * 8;
  return cover < resident ? (int)cover : resident;
}

// ---------------------------------------------------------------- geometry
// Spatial grid: m1 (x, fastest), m2 (y), m3 (z); unused dims are 1.
// Spectrum planes are padded: P_d = round_up(m_d, 64) for used dims, 1 otherwise.
struct Geometry {
  int dim = 1;
  int m1 = 1, m2 = 1, m3 = 1;
  int64_t m = 1;      // m1*m2*m3
  int P1 = 1, P2 = 1, P3 = 1;
  int64_t PS = 1;     // P1*P2*P3 (one real plane)
  int n = 2;          // time steps (power of two)
  int nh = 2;         // n/2 + 1 frequency blocks
  // time discretisation of L (eq. (pstepscheme), M = I): row k >= 2 reads
  // r0 u^k + r1 u^{k-1} + r2 u^{k-2} + tau K u^k; row 1 is a backward-Euler
  // step, u^1 + tau K u^1.  Backward Euler: (1, -1, 0); BDF2: (3/2, -2, 1/2).
  double r0 = 1.0, r1 = -1.0, r2 = 0.0;
  // spatial discretisation: finite differences (q1 = 0, M = I) or Q1 finite
  // elements on a uniform 2D grid (q1 = 1): 9-point M and tau K weights
  // qm = h^2/36 (16, 4, 1), qk = tau/3 (8, -1)
  int q1 = 0;
  double qm[3] = {0.0, 0.0, 0.0}, qk[2] = {0.0, 0.0};
};

// ---------------------------------------------------------------- launchers
// Each returns hipSuccess or the launch error.  Pointers are device pointers.

// y = L x (stencil + time bidiagonal), FP64.  c_d = tau / h_d^2.
hipError_t launch_apply_L(const Geometry& g, const double* x, double* y, double c1, double c2,
                          double c3, hipStream_t s);
// y = L x with the flux-form variable-coefficient operator; faces pre-scaled by tau/h^2.
// 2D with ay == nullptr: ax holds the four coupling planes [W, E, S, N][m2][m1]
// of a nonsymmetric five-point operator (node couples to its west, east, south,
// north neighbour with -W, -E, -S, -N, diagonal W + E + S + N), pre-scaled by tau.
hipError_t launch_apply_L_var(const Geometry& g, const double* x, double* y, const double* ax,
                              const double* ay, const double* az, hipStream_t s);

// Fused stencil passes (2D/3D only; AAO dim 1 uses the plain kernel).
// epi 1: partial sums of (f - L x)^2, one per block, y unused (may be null);
// epi 2: y = L x (not stored when y is null) and partial dots of L x with
// basis[0..q-1] (q <= kStencilDotsMax), q per block, (wsq non-null) partial
// sums of (L x)^2, one per block in wsq, and (w0sq non-null, q = 1 only)
// partial sums of basis[0]^2, one per block in w0sq.
// Constant coefficient: c1..c3 with ax = null; variable: ax, ay, az face weights.
// part must hold stencil_partials(g) * q doubles, wsq and w0sq stencil_partials(g).
constexpr int kStencilDotsMax = 4;
int64_t stencil_partials(const Geometry& g);
hipError_t launch_apply_L_epi(const Geometry& g, int epi, const double* x, double* y,
                              const double* f, const double* const* basis, int q, double* part,
                              double* wsq, double* w0sq, double c1, double c2, double c3,
                              const double* ax, const double* ay, const double* az,
                              hipStream_t s);

// Step 1: Gamma_eps scaling + forward time DFT (theta = e^{+2 pi i/n}) of a real
// [n][m] array into split re/im planes spec[k][2][PS], k = 0..n/2.
// gam[j] = eps^{j/n} / sqrt(n); tw = theta^e, e = 0..n-1.
hipError_t launch_time_fwd_f64(const Geometry& g, const double* x, double* spec,
                               const double* gam, const double* tw, hipStream_t s);
hipError_t launch_time_fwd_f32(const Geometry& g, const double* x, float* spec,
                               const float* gam, const float* tw, hipStream_t s);
// Step 3: Hermitian completion + inverse time DFT (theta^{-1}) + eps^{-j/n}/sqrt(n).
hipError_t launch_time_inv_f64(const Geometry& g, const double* spec, double* z,
                               const double* ginv, const double* tw, hipStream_t s);
hipError_t launch_time_inv_f32(const Geometry& g, const float* spec, double* z,
                               const float* ginv, const float* tw, hipStream_t s);

// Batched C[b] = A[b] * B[b] (row-major, all dims multiples of 64 except M which
// may be ragged).  Strides in elements; a zero stride broadcasts the operand.
hipError_t launch_gemm_f64(const double* A, int64_t sA, int lda, const double* B, int64_t sB,
                           int ldb, double* C, int64_t sC, int ldc, int M, int N, int K,
                           int batch, hipStream_t s);
hipError_t launch_gemm_f32(const float* A, int64_t sA, int lda, const float* B, int64_t sB,
                           int ldb, float* C, int64_t sC, int ldc, int M, int N, int K,
                           int batch, hipStream_t s);
// BF16 hi/lo split product: C = Ahi*Bhi + Ahi*Blo + Alo*Bhi, FP32 accumulate.
// A is given pre-split (Ahi, Alo as bf16 bit patterns); B is FP32 and split on load.
hipError_t launch_gemm_bf16x3(const uint16_t* Ahi, const uint16_t* Alo, int64_t sA, int lda,
                              const float* B, int64_t sB, int ldb, float* C, int64_t sC, int ldc,
                              int M, int N, int K, int batch, hipStream_t s);
// Same with the split operand on the right: C = A * S, A FP32 rows, S pre-split
// and symmetric (read row-wise), K = N.
hipError_t launch_gemm_bf16x3_right(const float* A, int64_t sA, int lda, const uint16_t* Bhi,
                                    const uint16_t* Blo, int64_t sB, int ldb, float* C,
                                    int64_t sC, int ldc, int M, int N, int K, int batch,
                                    hipStream_t s);

// Folded DST-I mode product over both planes of every frequency block (2D/3D).
// LEFT (axis y or z): each (k, plane, o) slab is a P x R-strided matrix whose
// rows run along the axis; RIGHT (axis x): each plane is P2*P3 rows of R = P1.
struct FoldArgs {
  int m;          // axis length m_d
  int Hp;         // P_d / 2 (multiple of 32): size of the folded tables
  int64_t R;      // stride between consecutive axis rows (LEFT) / data rows (RIGHT)
  int64_t PS;     // plane size
  int64_t OS;     // stride between outer slabs (LEFT axis y); 0 otherwise
  int nout;       // outer slabs per plane (P3 for LEFT axis y, else 1)
  int ndt;        // 64-wide data tiles per slab
  int nk;         // frequency blocks processed (n/2 + 1, or n/2 when packed)
  int packed;     // 1: block 0 pairs the real planes of frequencies 0 and n/2
  int axis;       // 0 = x, 1 = y, 2 = z
  int m1, m2, m3, P1, P2;
  // Q1 elements (2D, divide along y): the shifted divide also multiplies by
  // 1 / (mass eigenvalue along x (column) * along y (row)); null otherwise
  const double* ims_c = nullptr;
  const double* ims_r = nullptr;
};
// out = S_d applied along `axis`; Soe = S[0:h, 0::2], Soo = S[0:h, 1::2] (Hp x Hp,
// zero padded).  With lam != nullptr the result is divided by
// lambda_k + tmu1[i1] + tmu2[i2] + tmu3[i3] (tmu2/tmu3 may be null).
template <typename T>
hipError_t launch_dst_fold(const T* in, T* out, const T* Soe, const T* Soo, const FoldArgs& f,
                           bool left, const double* lam, const double* tmu1, const double* tmu2,
                           const double* tmu3, hipStream_t s);

// BF16x3 one-level fold (FP32 data): tabs = {hi(S_oe), lo(S_oe), hi(S_oo), lo(S_oo)},
// the BF16 splits of the FP32 folded tables; otherwise as launch_dst_fold.
hipError_t launch_dst_fold_bf16x3(const float* in, float* out, const uint16_t* const* tabs,
                                  const FoldArgs& f, bool left, const double* lam,
                                  const double* tmu1, const double* tmu2, const double* tmu3,
                                  hipStream_t s);

// Both in-plane DST-I products (x, then y) of every z slab of a 3D spectrum,
// in place, FP64, P1 = P2 = 128, odd m1, m2 in (64, 128] with the same
// second-fold quarter tables ([4][32][32]: A+, A-, B+, B-; equal m1 and m2).  Slabs: the nk frequency blocks' two planes (packed as in FoldArgs)
// times z < m3; padding must be zero on input and stays zero.
struct SlabArgs {
  int64_t PS;     // plane size (P1 P2 P3)
  int nk;         // frequency blocks processed
  int packed;     // 1: block 0 pairs the real planes of frequencies 0 and n/2
  int m1, m2, m3;
  int P1, P2, P3;
};
// FP64: tab = the [4][32][32] quarter tables as [tb][q][t]; FP32: the same
// tables in FP32, transposed to [tb][t][q].  m1 = m2 = 127 with tab3
// non-null: the third-fold products instead (tab3 = one 32 x 32 and six
// 16 x 16 tables, [q][kappa] each, in the order the kernel documents; FP64 or
// FP32 like the spectrum).
template <typename F>
hipError_t launch_dst_xy(F* spec, const F* tab, const SlabArgs& a, hipStream_t s,
                         const F* tab3 = nullptr);
// The last axis of a 3D FP64 spectrum (P1 = P2 = P3 = 128, m3 = 127) in one
// in-place pass on the third fold: forward product, shifted divide by
// lambda_k + tmu1[x] + tmu2[y] + tmu3[z] (lam as for launch_dst_fold), inverse
// product.  tab3 as for launch_dst_xy (the z axis' tables).  Slices: the nk
// blocks (packed as in SlabArgs) times y < m2 times two x halves; y rows
// >= m2 are not touched, padding elsewhere is zero on input and on output.
hipError_t launch_dst_zdiv(double* spec, const double* tab3, const SlabArgs& a,
                           const double* lam, const double* tmu1, const double* tmu2,
                           const double* tmu3, hipStream_t s);

// Two-level fold for odd m (P_d a multiple of 128): tabs = [4][Hq][Hq], Hq = P_d/4,
// the quarter tables A+, A-, B+, B- (rows q: output rows 2q for +, 2q+1 for -;
// columns: pair index t of the even (A) / odd (B) inputs).  Same arguments and
// result as launch_dst_fold.  Instantiated for FP64.
template <typename T>
hipError_t launch_dst_fold2(const T* in, T* out, const T* tabs, const FoldArgs& f, bool left,
                            const double* lam, const double* tmu1, const double* tmu2,
                            const double* tmu3, hipStream_t s);

// Forward product, shifted divide and inverse product along one LEFT axis (the
// last forward axis: y in 2D, z in 3D) in one kernel: FP64 or FP32 (the
// divide then in FP32), odd m, P_d = 128 or 256, f.ndt = columns / 16.  tt =
// the two-level fold tables transposed, [4][Hq][Hq] as [table][t][q], in the
// spectrum's type.  lam and tmu1..tmu3 as for the divide.
template <typename T>
hipError_t launch_dst_fold2_fused(const T* in, T* out, const T* tt, const FoldArgs& f,
                                  const double* lam, const double* tmu1, const double* tmu2,
                                  const double* tmu3, hipStream_t s);
// Two-level folded product along x (axis 0, no divide) with 16 whole rows per
// block, FP64, odd m, P1 = 128 or 256; f.ndt counts 16-row tiles per plane.
hipError_t launch_dst_fold2_rows(const double* in, double* out, const double* tt,
                                 const FoldArgs& f, hipStream_t s);

// Shifted divide in the doubly transformed domain:
// spec[k] <- spec[k] / (lambda_k + sum_d tmu_d[i_d]), complex, pads set to 0.
hipError_t launch_divide_f64(const Geometry& g, double* spec, const double* lam,
                             const double* tmu1, const double* tmu2, const double* tmu3,
                             hipStream_t s);
hipError_t launch_divide_f32(const Geometry& g, float* spec, const double* lam,
                             const double* tmu1, const double* tmu2, const double* tmu3,
                             hipStream_t s);

// Layout conversions for the step-by-step entry points (external spectrum
// layout: interleaved complex FP64 [nh][m][2]).
hipError_t launch_spec_to_ext(const Geometry& g, const void* spec, int is_f32, double* ext,
                              hipStream_t s);
hipError_t launch_ext_to_spec(const Geometry& g, const double* ext, void* spec, int is_f32,
                              hipStream_t s);

// ---------------------------------------------------------------- Krylov kernels
// Basis vectors: V_i = V + i*ldv, except V_0 = v0 when v0 is non-null.
// Partial dot products: part[b*q + i] = sum over block b's elements of V_i . w.
// krylov_blocks(len) blocks.  Then reduce_partials sums over blocks.
int krylov_blocks(int64_t len);
hipError_t launch_multidot(const double* V, int64_t ldv, const double* v0, int q,
                           const double* w, int64_t len, double* part, hipStream_t s);
// w -= sum_{i<q} h_i V_i, then mode 1: partial dots of V_i with the new w
// (q <= 8); mode 2: partial squared norm of the new w; mode 0: nothing.
hipError_t launch_axpy_dot(const double* V, int64_t ldv, const double* v0, int q,
                           const double* h, double* w, int64_t len, double* part, int mode,
                           hipStream_t s);
// out[i] (+)= scale[i] * sum over blocks (scale may be null: 1)
hipError_t launch_reduce_partials(const double* part, int nblk, int q, double* out,
                                  int accumulate, const double* scale, hipStream_t s);
// y = alpha * x with alpha a host scalar
hipError_t launch_scale_host(const double* x, double* y, int64_t len, double alpha, hipStream_t s);
// x = (set ? 0 : x) + sum_i c_i Z_i with c on device
hipError_t launch_multi_axpy(const double* Z, int64_t ldz, int q, const double* c, double* x,
                             int64_t len, int set, hipStream_t s);
// partial squared norm of (a - b) (b may be null -> ||a||^2)
hipError_t launch_diffnorm(const double* a, const double* b, int64_t len, double* part,
                           hipStream_t s);
// y = tau*f, y[0:m] += u0 (backward-Euler first step), y[m:2m] -= r2*u0 (the
// u^0 term of the second row of a two-step scheme; r2 = 0 for backward Euler)
hipError_t launch_build_rhs(const double* f, const double* u0, double* y, int64_t nm, int64_t m,
                            double tau, double r2, hipStream_t s);
// f[k] += the boundary couplings cb times the Dirichlet values gb[k] (2D):
// gb [n][2 m2 + 2 m1] = west (m2), east (m2), south (m1), north (m1) walls;
// cb the same layout without the time index.
hipError_t launch_boundary_source(const double* gb, const double* cb, double* f, int n, int m1,
                                  int m2, hipStream_t s);

// ---------------------------------------------------------------- multigrid (2D)
// One level's complex grid for all blocks: element (k, plane, j, i) at
// p + k*bstride + plane*pstride + j*pitch + i (elements of the level's type).
struct MgGrid {
  void* p = nullptr;
  int pitch = 0;
  int64_t pstride = 0, bstride = 0;
};
// Level couplings: face weights wx [m][m+1], wy [m+1][m], or, with wy == nullptr,
// the four coupling planes [W, E, S, N][m][m] in wx (all pre-scaled by tau).
// One smoothing step (red then black half sweep) in one launch from the old
// iterate e into eo (eo may be e only with zero_init: the old iterate is then
// zero and not read); with ec (coarse grid of mc points, 2 mc + 1 <= m) the
// old iterate is e + the bilinear interpolation of ec; with rc (coarse grid of
// mcr points, 2 mcr + 1 <= m), also rc = full-weighting restriction of
// r - B eo (rc aliases none of them).
template <typename T>
hipError_t mg_sweep(const MgGrid& e, const MgGrid& eo, const MgGrid& r, const MgGrid* rc,
                    int mcr, const MgGrid* ec, int mc, const void* wx, const void* wy,
                    const double* lam, int m, int nh, int zero_init, hipStream_t s);
template <typename T>
hipError_t mg_residual(const MgGrid& e, const MgGrid& r, const MgGrid& res, const void* wx,
                       const void* wy, const double* lam, int m, int nh, hipStream_t s);

// ---------------------------------------------------------------- learned correction
// Parameter vector: W1[C][3][3][3] G1[C][4] H1[C][4] W2[C][C][3][3] G2[C][4] H2[C][4]
// W3[2][C][3][3] b3[2] (float).
constexpr int kCnnC = 8;
constexpr int kCnnOffW1 = 0;
constexpr int kCnnOffG1 = kCnnOffW1 + kCnnC * 3 * 9;
constexpr int kCnnOffH1 = kCnnOffG1 + kCnnC * 4;
constexpr int kCnnOffW2 = kCnnOffH1 + kCnnC * 4;
constexpr int kCnnOffG2 = kCnnOffW2 + kCnnC * kCnnC * 9;
constexpr int kCnnOffH2 = kCnnOffG2 + kCnnC * 4;
constexpr int kCnnOffW3 = kCnnOffH2 + kCnnC * 4;
constexpr int kCnnOffB3 = kCnnOffW3 + 2 * kCnnC * 9;
constexpr int kCnnParams = kCnnOffB3 + 2;

int cnn_chunks(int HW);
int cnn_tiles(int H, int W);
hipError_t cnn_conv_fwd(int layer, const float* x, const float* w, const float* gam,
                        const float* bet, const float* bias, float* z, float* out, int B, int H,
                        int W, hipStream_t s);
hipError_t cnn_conv_bwd_data(int layer, const float* dz, const float* w, float* dx, int B, int H,
                             int W, hipStream_t s);
hipError_t cnn_conv_wgrad(int layer, const float* dz, const float* x, float* part, float* grad,
                          int B, int H, int W, hipStream_t s);
hipError_t cnn_film_bwd(const float* dh, const float* z, const float* h, const float* gam,
                        float* dz, float* part, float* dfilm, int B, int H, int W,
                        hipStream_t s);
hipError_t cnn_bias_grad(const float* dy, float* part, float* grad, int B, int H, int W,
                         hipStream_t s);
hipError_t cnn_film_params(const float* prm, const float* phi, float* gb, int B, hipStream_t s);
// phi[b] = (Re lambda_b, Im lambda_b, log|lambda_b|, 1) from lambda [B][2] (FP64, device)
hipError_t cnn_features(const double* lam, float* phi, int B, hipStream_t s);
hipError_t cnn_film_grad(const float* dfilm, const float* phi, float* grad, int B, int layer,
                         hipStream_t s);
hipError_t cnn_resid_loss(const float* y, const float* rho, const float* rn, const float* phi,
                          const float* wx, const float* wy, float* E, float* Q, float* G,
                          float* Hb, float* dy, float* part, float* lb, float* out, int B, int H,
                          int W, hipStream_t s);
hipError_t cnn_adam(float* prm, const float* g, float* m, float* v, int np, float lr, int step,
                    hipStream_t s);
hipError_t cnn_gather(const float* px, const float* pphi, const float* ptn, const float* loga,
                      const int* idx, float* X, float* R, float* phi, float* tn, int B, int HW,
                      hipStream_t s);
template <typename T>
hipError_t cnn_block_sumsq(const MgGrid& v, int m, int nh, float* part, float* out, hipStream_t s);
template <typename T>
hipError_t cnn_pack_input(const MgGrid& v, const float* ss, const float* loga, float* X, int m,
                          int nh, int nch, hipStream_t s);
// vo = v + s Y / (lambda + d) per block (vo may be v)
template <typename T>
hipError_t cnn_unpack_add(const float* Y, const float* ss, const MgGrid& v, const MgGrid& vo,
                          const double* lam, const float* wx, const float* wy, int m, int nh,
                          hipStream_t s);

}  // namespace aao
